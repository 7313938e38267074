"""MI355X (gfx950) per-cluster RANSAC velocity and heading estimator.

Singh, Sil, Sharma, "Parallelized Instantaneous Velocity and Heading Estimation
of Objects using Single Imaging Radar": RANSAC over the radar velocity profile
(Sec. 3.1, Alg. 1), least-squares refit on the inliers (Sec. 3.2, Eq. 7,
Alg. 2) and heading (Eq. 8), as hand-written HIP kernels behind a C ABI
(include/rv.h).  The entry points below mirror the C names; importing this
package does not load the library, calling an entry point does (and fails
loudly when it has not been built).
"""
from importlib import import_module

_BINDING_NAMES = (
    "rv_estimate_velocity", "rv_workspace_bytes", "rv_last_error", "rv_stage_timing",
    "rv_stage_times", "rv_philox4x32_10", "allocate_outputs", "load_library", "RVError",
    "rv_tuning_default", "rv_batch_workspace_bytes", "rv_estimate_velocity_batch",
    "rv_graph_capture_batch", "allocate_batch_outputs", "RVTuning", "RVGraph",
    "RVServer", "RVServerConfig", "rv_server_config_default", "rv_server_frame_bytes",
    "rv_estimate_velocity_paper", "rv_paper_workspace_bytes", "rv_estimate_velocity_part",
    "rv_estimate_velocity_pipelined", "rv_estimate_velocity_noalloc",
    "host_device_pointer", "PreparedEstimate", "estimate_velocity",
)

__all__ = list(_BINDING_NAMES)


def __getattr__(name):
    if name in _BINDING_NAMES:
        return getattr(import_module(".binding", __name__), name)
    raise AttributeError(name)
