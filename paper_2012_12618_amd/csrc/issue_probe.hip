// issue_probe.hip -- wave64 issue rates of the instructions the scoring loops
// are made of, on the current device at full occupancy (eight waves per SIMD).
//
// Each kernel runs ITER iterations of 16 independent copies of one instruction
// (or of one scoring row: the float32 row of the estimator, two v_fma_f32 and a
// compare whose 64-lane mask the scalar unit popcounts, and the FP16 row, one
// v_dot2_f32_f16 and a compare), and of the hypothesis generation's integer
// and FP64 instructions.  The only memory access is one store per
// thread into an array of grid x block words.  Prints one JSON object: for each
// case the kernel time, wave64 vector instructions per SIMD-cycle and
// SIMD-cycles per instruction, scalar instructions per CU-cycle, and CU-cycles
// per 64-lane row (at 2.4 GHz, the clock the chip holds under this load).
//
// Built by paper_2012_12618_amd/build.py into _lib/issue_probe; run by
// `bench.py --workload issue-rates`.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>

namespace {

constexpr int kIter = 2048;
constexpr int kBlock = 256;
typedef uint32_t u32;
typedef uint64_t u64;

#define RV_PROBE_16(STMT) _Pragma("unroll") for (int i = 0; i < 16; ++i) { STMT; }

__global__ __launch_bounds__(kBlock) void k_fma(float *out, float a, float b) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_fma_f32 %0, %1, %2, %0" : "+v"(x[i]) : "v"(a), "v"(b)))
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_add_u32(float *out, u32 a) {
    u32 x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_add_u32 %0, %1, %0" : "+v"(x[i]) : "v"(a)))
    }
    u32 s = 0;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = (float)s;
}

__global__ __launch_bounds__(kBlock) void k_max(float *out, float t) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_max_f32 %0, %1, %0" : "+v"(x[i]) : "v"(t)))
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_cmp_abs_sgpr(float *out, float t) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    u64 acc = 0;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(u64 m; asm volatile("v_cmp_lt_f32_e64 %0, |%1|, %2" : "=s"(m) : "v"(x[i]), "v"(t));
                    if (i == 15) acc ^= m)
    }
    out[blockIdx.x * kBlock + threadIdx.x] = (float)(acc & 0xFF);
}

__global__ __launch_bounds__(kBlock) void k_cmp_vcc(float *out, float t) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_cmp_lt_f32_e32 vcc, %0, %1" : : "v"(x[i]), "v"(t) : "vcc"))
    }
    out[blockIdx.x * kBlock + threadIdx.x] = x[3];
}

__global__ __launch_bounds__(kBlock) void k_dot2(float *out, u32 a, u32 b) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_dot2_f32_f16 %0, %1, %2, %0" : "+v"(x[i]) : "v"(a), "v"(b)))
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_dot2c(float *out, u32 a, u32 b) {
    float x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001f + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_dot2c_f32_f16 %0, %1, %2" : "+v"(x[i]) : "v"(a), "v"(b)))
    }
    float s = 0.0f;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_pk_fma_f16(float *out, u32 a, u32 b) {
    u32 x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_pk_fma_f16 %0, %1, %2, %0" : "+v"(x[i]) : "v"(a), "v"(b)))
    }
    u32 s = 0;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = (float)s;
}

// Scalar unit: s_bcnt1_i32_b64 + s_add_i32 (the popcount and accumulation of
// one row's mask), four independent chains.
__global__ __launch_bounds__(kBlock) void k_salu(float *out, u64 m0) {
    u32 c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    const u64 m = m0 ^ blockIdx.x;
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            u32 t0, t1, t2, t3;
            asm volatile(
                "s_bcnt1_i32_b64 %0, %8\n\ts_bcnt1_i32_b64 %1, %8\n\t"
                "s_bcnt1_i32_b64 %2, %8\n\ts_bcnt1_i32_b64 %3, %8\n\t"
                "s_add_i32 %4, %4, %0\n\ts_add_i32 %5, %5, %1\n\t"
                "s_add_i32 %6, %6, %2\n\ts_add_i32 %7, %7, %3"
                : "=&s"(t0), "=&s"(t1), "=&s"(t2), "=&s"(t3), "+s"(c0), "+s"(c1), "+s"(c2), "+s"(c3)
                : "s"(m)
                : "scc");
        }
    }
    out[blockIdx.x * kBlock + threadIdx.x] = (float)(c0 + c1 + c2 + c3);
}

// The float32 scoring row as the compiler builds it (two FMAs, a compare into
// a 64-lane mask, popcount and add on the scalar unit), 16 rows per hypothesis.
__global__ __launch_bounds__(kBlock) void k_row_f32(float *out, float hx, float hy, float t) {
    float c[16], s[16], v[16];
    for (int i = 0; i < 16; ++i) {
        c[i] = 0.5f + i * 0.01f;
        s[i] = 0.3f;
        v[i] = threadIdx.x * 0.01f + i;
    }
    u32 n = 0;
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const float e = __builtin_fmaf(-hy, s[r], __builtin_fmaf(-hx, c[r], v[r]));
            n += (u32)__builtin_popcountll(__builtin_amdgcn_ballot_w64(__builtin_fabsf(e) < t));
        }
        hx += 1e-7f;
    }
    out[blockIdx.x * kBlock + threadIdx.x] = (float)n;
}

// The FP16 scoring row: v_dot2_f32_f16 and a compare, four rows per asm block
// (each compare three instructions after the dot product it reads).
__global__ __launch_bounds__(kBlock) void k_row_f16(float *out, u32 nd, float t) {
    u32 c[16];
    float w[16];
    for (int i = 0; i < 16; ++i) {
        c[i] = 0x3C003800u + i;
        w[i] = threadIdx.x * 0.01f + i;
    }
    u32 n = 0;
    for (int it = 0; it < kIter; ++it) {
#pragma unroll
        for (int r = 0; r < 16; r += 4) {
            float e0, e1, e2, e3;
            u64 m0, m1, m2, m3;
            asm volatile(
                "v_dot2_f32_f16 %0, %8, %12, %14\n\tv_dot2_f32_f16 %1, %9, %12, %15\n\t"
                "v_dot2_f32_f16 %2, %10, %12, %16\n\tv_dot2_f32_f16 %3, %11, %12, %17\n\t"
                "v_cmp_lt_f32_e64 %4, |%0|, %13\n\tv_cmp_lt_f32_e64 %5, |%1|, %13\n\t"
                "v_cmp_lt_f32_e64 %6, |%2|, %13\n\tv_cmp_lt_f32_e64 %7, |%3|, %13"
                : "=&v"(e0), "=&v"(e1), "=&v"(e2), "=&v"(e3), "=s"(m0), "=s"(m1), "=s"(m2),
                  "=s"(m3)
                : "v"(c[r]), "v"(c[r + 1]), "v"(c[r + 2]), "v"(c[r + 3]), "v"(nd), "v"(t),
                  "v"(w[r]), "v"(w[r + 1]), "v"(w[r + 2]), "v"(w[r + 3]));
            n += (u32)(__builtin_popcountll(m0) + __builtin_popcountll(m1) +
                       __builtin_popcountll(m2) + __builtin_popcountll(m3));
        }
        nd += 1;
    }
    out[blockIdx.x * kBlock + threadIdx.x] = (float)n;
}

// The integer and FP64 instructions of a hypothesis's generation: the
// 32x32->64 multiply-add of each Philox round, a 32-bit high product, and the
// FP64 fused multiply-add of the seed solve.
__global__ __launch_bounds__(kBlock) void k_mad_u64(float *out, u32 a) {
    u64 x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(u64 carry; asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0"
                                            : "+v"(x[i]), "=s"(carry) : "v"((u32)x[i]), "v"(a)))
    }
    u64 s = 0;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = (float)(s & 0xFFFF);
}

__global__ __launch_bounds__(kBlock) void k_mul_hi_u32(float *out, u32 a) {
    u32 x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_mul_hi_u32 %0, %1, %0" : "+v"(x[i]) : "v"(a)))
    }
    u32 s = 0;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = (float)s;
}

__global__ __launch_bounds__(kBlock) void k_fma_f64(float *out, double a, double b) {
    double x[16];
    for (int i = 0; i < 16; ++i) x[i] = threadIdx.x * 0.001 + i;
    for (int it = 0; it < kIter; ++it) {
        RV_PROBE_16(asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(x[i]) : "v"(a), "v"(b)))
    }
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += x[i];
    out[blockIdx.x * kBlock + threadIdx.x] = (float)s;
}

struct Case {
    const char *name;
    int valu_per_iter, salu_per_iter, rows_per_iter;
};

const Case kCases[] = {
    {"v_fma_f32", 16, 0, 0},
    {"v_add_u32", 16, 0, 0},
    {"v_max_f32", 16, 0, 0},
    {"v_cmp_lt_f32_e64 |x| -> SGPR pair", 16, 0, 0},
    {"v_cmp_lt_f32_e32 -> VCC", 16, 0, 0},
    {"v_dot2_f32_f16 (VOP3P)", 16, 0, 0},
    {"v_dot2c_f32_f16 (VOP2)", 16, 0, 0},
    {"v_pk_fma_f16", 16, 0, 0},
    {"s_bcnt1_i32_b64 + s_add_i32", 0, 32, 0},
    {"float32 row: 2 v_fma_f32 + v_cmp | s_bcnt1 + s_add", 48, 32, 16},
    {"FP16 row: v_dot2_f32_f16 + v_cmp | s_bcnt1 + s_add", 32, 32, 16},
    {"v_mad_u64_u32", 16, 0, 0},
    {"v_mul_hi_u32", 16, 0, 0},
    {"v_fma_f64", 16, 0, 0},
};

hipError_t launch(int which, unsigned grid, float *out) {
    const dim3 g(grid), b(kBlock);
    switch (which) {
        case 0: hipLaunchKernelGGL(k_fma, g, b, 0, 0, out, 1.0001f, 1e-7f); break;
        case 1: hipLaunchKernelGGL(k_add_u32, g, b, 0, 0, out, 3u); break;
        case 2: hipLaunchKernelGGL(k_max, g, b, 0, 0, out, 3.0f); break;
        case 3: hipLaunchKernelGGL(k_cmp_abs_sgpr, g, b, 0, 0, out, 3.0f); break;
        case 4: hipLaunchKernelGGL(k_cmp_vcc, g, b, 0, 0, out, 3.0f); break;
        case 5: hipLaunchKernelGGL(k_dot2, g, b, 0, 0, out, 0x3C003C00u, 0x00010001u); break;
        case 6: hipLaunchKernelGGL(k_dot2c, g, b, 0, 0, out, 0x3C003C00u, 0x00010001u); break;
        case 7: hipLaunchKernelGGL(k_pk_fma_f16, g, b, 0, 0, out, 0x3C003C00u, 0x00010001u); break;
        case 8: hipLaunchKernelGGL(k_salu, g, b, 0, 0, out, 0x123456789ABCDEFull); break;
        case 9: hipLaunchKernelGGL(k_row_f32, g, b, 0, 0, out, 0.1f, 0.2f, 0.15f); break;
        case 10: hipLaunchKernelGGL(k_row_f16, g, b, 0, 0, out, 0x00010001u, 0.15f); break;
        case 11: hipLaunchKernelGGL(k_mad_u64, g, b, 0, 0, out, 0xD2511F53u); break;
        case 12: hipLaunchKernelGGL(k_mul_hi_u32, g, b, 0, 0, out, 0xCD9E8D57u); break;
        case 13: hipLaunchKernelGGL(k_fma_f64, g, b, 0, 0, out, 1.0000001, 1e-9); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

#define RV_PROBE_CHECK(x)                                                                     \
    do {                                                                                      \
        const hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                               \
            fprintf(stderr, "issue_probe: %s failed: %s\n", #x, hipGetErrorString(e_));     \
            return 1;                                                                         \
        }                                                                                     \
    } while (0)

int main() {
    int dev = 0, cus = 0;
    RV_PROBE_CHECK(hipGetDevice(&dev));
    RV_PROBE_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipDeviceProp_t prop;
    RV_PROBE_CHECK(hipGetDeviceProperties(&prop, dev));
    const unsigned grid = (unsigned)cus * 8u;  // four waves per block: eight waves per SIMD
    float *out = nullptr;
    RV_PROBE_CHECK(hipMalloc(&out, (size_t)grid * kBlock * sizeof(float)));
    hipEvent_t e0, e1;
    RV_PROBE_CHECK(hipEventCreate(&e0));
    RV_PROBE_CHECK(hipEventCreate(&e1));
    const double clock_hz = 2.4e9;
    const double waves = (double)grid * (kBlock / 64);
    printf("{\"device\": \"%s\", \"compute_units\": %d, \"waves_per_simd\": 8, \"iterations\": %d, "
           "\"clock_ghz_assumed\": 2.4, \"cases\": [",
           prop.gcnArchName, cus, kIter);
    const int n_cases = (int)(sizeof kCases / sizeof kCases[0]);
    for (int w = 0; w < n_cases; ++w) {
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {  // the first launch warms the clock up
            RV_PROBE_CHECK(hipEventRecord(e0, 0));
            RV_PROBE_CHECK(launch(w, grid, out));
            RV_PROBE_CHECK(hipEventRecord(e1, 0));
            RV_PROBE_CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            RV_PROBE_CHECK(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0 && ms < best) best = ms;
        }
        const Case &c = kCases[w];
        const double cycles = best * 1e-3 * clock_hz;
        const double valu = waves * kIter * c.valu_per_iter, salu = waves * kIter * c.salu_per_iter;
        const double rows = waves * kIter * c.rows_per_iter;
        printf("%s{\"case\": \"%s\", \"kernel_ms\": %.4f, \"valu_per_simd_cycle\": %.4f, "
               "\"simd_cycles_per_valu\": %.3f, \"salu_per_cu_cycle\": %.4f, "
               "\"cu_cycles_per_row\": %.4f}",
               w ? ", " : "", c.name, best, valu / (cus * 4.0 * cycles),
               valu > 0 ? cus * 4.0 * cycles / valu : 0.0, salu / (cus * cycles),
               rows > 0 ? cycles * cus / rows : 0.0);
    }
    printf("]}\n");
    RV_PROBE_CHECK(hipFree(out));
    return 0;
}
