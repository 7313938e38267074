// rv_cli.cpp -- the estimator from a plain C/C++ program, through the C ABI of
// include/rv.h only (no Python, no torch): reads one CSR frame from raw files,
// estimates it on the current GPU and writes the per-cluster results as raw
// files.
//
//   rv_cli THETA VD OFFSETS N_HYP TAU SEED OUT_PREFIX
//
//   THETA, VD    float32 little-endian arrays of the frame's points (azimuth in
//                radians, radial Doppler velocity in m/s), same length N.
//   OFFSETS      int32 array of K + 1 cluster offsets (0, ..., N).
//   N_HYP, TAU, SEED  hypotheses per cluster, inlier threshold (m/s), Philox key.
//   OUT_PREFIX   writes OUT_PREFIX.vx, .vy, .heading (float32 [K]), .n_inliers
//                (int32 [K]) and .status (uint8 [K]).
//
// Prints one line, "clusters K points N ok M", M the clusters with status
// RV_CLUSTER_OK, and exits 0; on an error it prints the library's or the HIP
// runtime's message and exits 1.  Built by paper_2012_12618_amd/build.py into
// _lib/rv_cli (linked against _lib/librv.so).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "rv.h"

namespace {

// Reads a whole file of T elements; returns false on any error.
template <typename T>
bool read_file(const char *path, std::vector<T> &out) {
    FILE *f = fopen(path, "rb");
    if (f == nullptr) return false;
    bool ok = fseek(f, 0, SEEK_END) == 0;
    const long bytes = ok ? ftell(f) : -1;
    ok = ok && bytes >= 0 && bytes % (long)sizeof(T) == 0 && fseek(f, 0, SEEK_SET) == 0;
    if (ok) {
        out.resize((size_t)bytes / sizeof(T));
        ok = fread(out.data(), sizeof(T), out.size(), f) == out.size();
    }
    fclose(f);
    return ok;
}

template <typename T>
bool write_file(const char *prefix, const char *suffix, const std::vector<T> &data) {
    char path[4096];
    if (snprintf(path, sizeof path, "%s.%s", prefix, suffix) >= (int)sizeof path) return false;
    FILE *f = fopen(path, "wb");
    if (f == nullptr) return false;
    const bool ok = fwrite(data.data(), sizeof(T), data.size(), f) == data.size();
    return (fclose(f) == 0) && ok;
}

bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    fprintf(stderr, "rv_cli: %s failed: %s\n", what, hipGetErrorString(e));
    return false;
}

// Device copy of a host array (nullptr for an empty one).
template <typename T>
bool to_device(const std::vector<T> &h, T **d) {
    *d = nullptr;
    if (h.empty()) return true;
    return hip_ok(hipMalloc((void **)d, h.size() * sizeof(T)), "hipMalloc") &&
           hip_ok(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice),
                  "hipMemcpy to the device");
}

template <typename T>
bool to_host(const T *d, std::vector<T> &h) {
    if (h.empty()) return true;
    return hip_ok(hipMemcpy(h.data(), d, h.size() * sizeof(T), hipMemcpyDeviceToHost),
                  "hipMemcpy to the host");
}

int run(int argc, char **argv) {
    if (argc != 8) {
        fprintf(stderr, "usage: %s THETA VD OFFSETS N_HYP TAU SEED OUT_PREFIX\n", argv[0]);
        return 1;
    }
    std::vector<float> theta, vd;
    std::vector<int32_t> off;
    if (!read_file(argv[1], theta) || !read_file(argv[2], vd) || !read_file(argv[3], off)) {
        fprintf(stderr, "rv_cli: cannot read the input files\n");
        return 1;
    }
    if (theta.size() != vd.size() || off.empty()) {
        fprintf(stderr, "rv_cli: THETA and VD differ in length, or OFFSETS is empty\n");
        return 1;
    }
    const int64_t n_points = (int64_t)theta.size(), n_clusters = (int64_t)off.size() - 1;
    const int32_t n_hyp = (int32_t)strtol(argv[4], nullptr, 10);
    const float tau = strtof(argv[5], nullptr);
    const uint64_t seed = strtoull(argv[6], nullptr, 0);

    float *d_theta = nullptr, *d_vd = nullptr, *d_vx = nullptr, *d_vy = nullptr;
    float *d_heading = nullptr;
    int32_t *d_off = nullptr, *d_n_in = nullptr;
    uint8_t *d_status = nullptr;
    void *d_ws = nullptr;
    const size_t ws_bytes = rv_workspace_bytes(n_clusters, n_points, n_hyp);
    const size_t K = (size_t)n_clusters;
    bool ok = to_device(theta, &d_theta) && to_device(vd, &d_vd) && to_device(off, &d_off);
    if (ok && K > 0)
        ok = hip_ok(hipMalloc((void **)&d_vx, K * sizeof(float)), "hipMalloc") &&
             hip_ok(hipMalloc((void **)&d_vy, K * sizeof(float)), "hipMalloc") &&
             hip_ok(hipMalloc((void **)&d_heading, K * sizeof(float)), "hipMalloc") &&
             hip_ok(hipMalloc((void **)&d_n_in, K * sizeof(int32_t)), "hipMalloc") &&
             hip_ok(hipMalloc((void **)&d_status, K), "hipMalloc");
    if (ok && ws_bytes > 0) ok = hip_ok(hipMalloc(&d_ws, ws_bytes), "hipMalloc");
    hipStream_t stream = nullptr;
    if (ok) ok = hip_ok(hipStreamCreate(&stream), "hipStreamCreate");
    if (ok) {
        const int rc = rv_estimate_velocity(d_theta, d_vd, d_off, n_clusters, n_points, n_hyp, tau,
                                            seed, d_vx, d_vy, d_heading, d_n_in, d_status, nullptr,
                                            nullptr, nullptr, nullptr, d_ws, ws_bytes, stream);
        if (rc != RV_OK) {
            fprintf(stderr, "rv_cli: rv_estimate_velocity returned %d: %s\n", rc, rv_last_error());
            ok = false;
        }
    }
    if (ok) ok = hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize");
    std::vector<float> vx(K), vy(K), heading(K);
    std::vector<int32_t> n_in(K);
    std::vector<uint8_t> status(K);
    if (ok)
        ok = to_host(d_vx, vx) && to_host(d_vy, vy) && to_host(d_heading, heading) &&
             to_host(d_n_in, n_in) && to_host(d_status, status);
    if (ok) {
        ok = write_file(argv[7], "vx", vx) && write_file(argv[7], "vy", vy) &&
             write_file(argv[7], "heading", heading) && write_file(argv[7], "n_inliers", n_in) &&
             write_file(argv[7], "status", status);
        if (!ok) fprintf(stderr, "rv_cli: cannot write the output files\n");
    }
    if (stream != nullptr) (void)hipStreamDestroy(stream);
    void *bufs[] = {d_theta, d_vd, d_off, d_vx, d_vy, d_heading, d_n_in, d_status, d_ws};
    for (void *p : bufs)
        if (p != nullptr) (void)hipFree(p);
    if (!ok) return 1;
    int64_t n_ok = 0;
    for (uint8_t s : status) n_ok += s == RV_CLUSTER_OK;
    printf("clusters %lld points %lld ok %lld\n", (long long)n_clusters, (long long)n_points,
           (long long)n_ok);
    return 0;
}

}  // namespace

int main(int argc, char **argv) { return run(argc, argv); }
