// Device-side helpers shared by the ICWF kernels: complex arithmetic on
// double2 / float2, the model interactions, and the kernel-argument structs.
//
// Model interactions (Eq. 2 with no vector potential).  The library splits the
// full interaction into one-coordinate parts and a coupling part,
//     W(r, R) = V_1(r) + V_2(R) + W_c(r, R),
// Shin-Metiu:  V_1 = -g(r - L/2; R_r) - g(r + L/2; R_l)
//              V_2 = 1/|L/2 - R| + 1/|L/2 + R|
//              W_c = -g(r - R; R_f),          g(x; a) = erf(|x|/a)/|x|
// cavity:      V_1 = -depth/sqrt(x^2 + a^2),  V_2 = omega^2 q^2/2,  W_c = lam q x.
// The propagators use the full W; the Eq. 8 coupling matrix is assembled from
// W_c only plus a column scaling of S (the one-coordinate parts cancel between
// Eq. 9b and Eqs. 9c-9d except at the ket's own trajectory).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icwf {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;

struct ModelParams {
    int32_t kind;      // 1 = Shin-Metiu, 2 = cavity
    double p[8];
};

__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// conj(a) * b in FP32
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// g(x; a) = erf(|x|/a)/|x| with its limit 2/(sqrt(pi) a) at x = 0 (Taylor
// series 2/(sqrt(pi) a)(1 - z^2/3 + z^4/10) below |x| < 1e-4 a, z = x/a).
__device__ inline double erf_over_x(double x, double a) {
    double ax = fabs(x);
    double z = ax / a;
    if (z < 1e-4) {
        double z2 = z * z;
        return kTwoOverSqrtPi / a * (1.0 - z2 / 3.0 + z2 * z2 / 10.0);
    }
    return erf(z) / ax;
}

// V_1 at a point of species 1.
__device__ inline double model_v1(const ModelParams &m, double r) {
    if (m.kind == 1) {
        double half = 0.5 * m.p[0];
        return -erf_over_x(r - half, m.p[3]) - erf_over_x(r + half, m.p[2]);
    }
    return -m.p[0] / sqrt(r * r + m.p[1] * m.p[1]);
}

// V_2 at a point of species 2.
__device__ inline double model_v2(const ModelParams &m, double R) {
    if (m.kind == 1) {
        double half = 0.5 * m.p[0];
        return 1.0 / fabs(half - R) + 1.0 / fabs(half + R);
    }
    return 0.5 * m.p[2] * m.p[2] * R * R;
}

// Coupling part W_c(r, R).
__device__ inline double model_wc(const ModelParams &m, double r, double R) {
    if (m.kind == 1) return -erf_over_x(r - R, m.p[1]);
    return m.p[3] * R * r;
}

// Full interaction W(r, R).
__device__ inline double model_w(const ModelParams &m, double r, double R) {
    return model_v1(m, r) + model_v2(m, R) + model_wc(m, r, R);
}

// Result layout of the 16 x 16 x 4 matrix-core products on gfx950: lane l,
// accumulator register v holds column l % 16 and row
//   (l / 16) + 4 v      for v_mfma_f64_16x16x4_f64,
//   4 (l / 16) + v      for v_mfma_f32_16x16x4_f32.
// (Operands: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] for both.)
__device__ inline int mfma_row_f64(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ inline int mfma_row_f32(int lane, int v) { return 4 * (lane >> 4) + v; }
__device__ inline int mfma_row(double, int lane, int v) { return mfma_row_f64(lane, v); }
__device__ inline int mfma_row(float, int lane, int v) { return mfma_row_f32(lane, v); }

// Batched launches (several simulations of one shape in one launch): the
// simulation blockIdx.z (the outer part of it where z has another use) finds
// every buffer at the address of the launch's first simulation plus
// zoff[blockIdx.z] bytes, its workspace being laid out the same way.
// zoff == nullptr: one simulation, no offset.
__device__ inline long long batch_offset(const long long *zoff, int z) { return zoff ? zoff[z] : 0; }
__device__ inline long long batch_offset(const long long *zoff) { return batch_offset(zoff, blockIdx.z); }
template <typename T>
__device__ inline T *zshift(T *p, long long o) {
    return p ? reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) + static_cast<uintptr_t>(o)) : p;
}

// Device status flags (one int32 each, in the workspace).
enum Flag : int32_t { kFlagHalt = 0, kFlagNode = 1, kFlagSolve = 2, kFlagNonfinite = 3, kFlagOut = 4,
                      kFlagHang = 5, kNumFlags = 8 };

// Bounded wait of one thread for an int32 flag written by another
// work-group (agent-scope acquire).  Every wait ends: after ~2^22 polls it
// raises kFlagHang and kFlagHalt and returns false, and the caller goes on
// with whatever is in memory (the host then reports the error).
__device__ inline bool wait_flag(const int32_t *flag, int32_t *status) {
    for (int it = 0; it < (1 << 22); ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    atomicOr(&status[kFlagHang], 1);
    atomicOr(&status[kFlagHalt], 1);
    return false;
}

__device__ inline void set_flag(int32_t *flag) {
    __hip_atomic_store(flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace icwf
