// Hermitian-CWF propagation (Eqs. 5-6 with the eta potentials reduced to a
// dropped phase): every conditional wavefunction takes one Strang
// split-operator step under its own conditioned potential, the conditioning
// coordinate frozen at the step's start:
//     psi <- e^{-i V dt/2} IFFT[ e^{-i k^2 dt/2m} FFT( e^{-i V dt/2} psi ) ],
//     V_1^a(r_i) = W(r_i, R^a),   V_2^a(R_j) = W(r^a, R_j).
//
// One work-group per CWF.  The CWF is read once from HBM (coalesced), stays in
// LDS through both FFTs (Stockham autosort, radix 4 with one radix-2 pass for
// odd log2 n, twiddles from a table), and is written once.  The potential
// phase is evaluated once per point (one erf, one sincos) and kept in
// registers for both half steps.  The inverse FFT is the forward one applied
// to the conjugate.  Bound: HBM (2 x 16 bytes per grid point per step).
#include "icwf_plan.hpp"

namespace icwf {

namespace {

constexpr int kMaxPts = 4;   // points per thread (threads = max(64, n/4))

__device__ inline void radix4(double2 &a0, double2 &a1, double2 &a2, double2 &a3) {
    double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    double2 x1 = make_double2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
    double2 x3 = make_double2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
    a1 = x1;
    a3 = x3;
}

// One Stockham pass of radix R (2 or 4) with Ns the size of the sub-transforms
// already done.  Butterfly j reads sh[j + r n/R], twiddles by
// exp(-2 pi i r k / (Ns R)) with k = j mod Ns, and writes
// sh[(j - k) R + k + r Ns].  All reads happen before the barrier, all writes
// after it, so one LDS buffer suffices.
template <int R>
__device__ inline void stockham_pass(double2 *sh, int n, int Ns, const double2 *__restrict__ tw, int T,
                                     int tid) {
    constexpr int kMaxBf = 2;   // butterflies per thread: n/R <= 2 T
    double2 v[kMaxBf][R];
    const int nbf = n / R;
    const int st = n / (Ns * R);
#pragma unroll
    for (int b = 0; b < kMaxBf; ++b) {
        const int j = tid + b * T;
        if (j < nbf) {
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = sh[j + r * nbf];
#pragma unroll
            for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[(r * k * st) & (n - 1)]);
            if (R == 4) {
                radix4(v[b][0], v[b][1], v[b][2], v[b][3]);
            } else {
                const double2 a = v[b][0], c = v[b][1];
                v[b][0] = cadd(a, c);
                v[b][1] = csub(a, c);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kMaxBf; ++b) {
        const int j = tid + b * T;
        if (j < nbf) {
            const int k = j & (Ns - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) sh[base + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

__device__ inline void fft_forward(double2 *sh, int n, int log2n, const double2 *__restrict__ tw, int T,
                                   int tid) {
    int Ns = 1;
    if (log2n & 1) {
        stockham_pass<2>(sh, n, Ns, tw, T, tid);
        Ns = 2;
    }
    while (Ns < n) {
        stockham_pass<4>(sh, n, Ns, tw, T, tid);
        Ns *= 4;
    }
}

__global__ void k_propagate(double2 *__restrict__ psi, int n, int log2n, const double *__restrict__ vstat,
                            double x_min, double h, const double *__restrict__ cond, int species,
                            ModelParams mp, const double2 *__restrict__ kin, const double2 *__restrict__ tw,
                            double dt, float2 *__restrict__ psi_f32, const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    extern __shared__ double2 sh[];
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    double2 *p = psi + (size_t)blockIdx.x * n;
    const double c = cond[blockIdx.x];
    // part of the conditioned potential that is constant on this CWF's grid
    const double vconst = (species == 1) ? model_v2(mp, c) : model_v1(mp, c);

    double2 ph[kMaxPts];
#pragma unroll
    for (int q = 0; q < kMaxPts; ++q) {
        const int i = tid + q * T;
        if (i < n) {
            const double x = x_min + i * h;
            const double V = vstat[i] + vconst + ((species == 1) ? model_wc(mp, x, c) : model_wc(mp, c, x));
            double s, co;
            sincos(-0.5 * dt * V, &s, &co);
            ph[q] = make_double2(co, s);
            sh[i] = cmul(ph[q], p[i]);
        }
    }
    __syncthreads();
    fft_forward(sh, n, log2n, tw, T, tid);
    for (int i = tid; i < n; i += T) sh[i] = cconj(cmul(kin[i], sh[i]));
    __syncthreads();
    fft_forward(sh, n, log2n, tw, T, tid);
    const double inv_n = 1.0 / n;
#pragma unroll
    for (int q = 0; q < kMaxPts; ++q) {
        const int i = tid + q * T;
        if (i < n) {
            const double2 v = cmul(ph[q], cscale(cconj(sh[i]), inv_n));
            p[i] = v;
            // FP32 copy for the mixed form's FP32 contraction
            if (psi_f32) psi_f32[(size_t)blockIdx.x * n + i] = make_float2((float)v.x, (float)v.y);
        }
    }
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

void launch_propagate(const Dims &d, const Bufs &b, int species, hipStream_t s) {
    const int n = species == 1 ? d.nr : d.nR;
    const int T = n / 4 < 64 ? 64 : n / 4;
    const size_t lds = sizeof(double2) * n;
    if (species == 1) {
        hipLaunchKernelGGL(k_propagate, dim3(d.N), dim3(T), lds, s, b.psi1, n, ilog2(n), b.vstat_r, d.r_min,
                           d.hr, b.R, 1, d.mp, b.kin_r, b.tw_r, d.dt, d.prec == 1 ? b.psi1_f32 : nullptr,
                           b.flags);
    } else {
        hipLaunchKernelGGL(k_propagate, dim3(d.N), dim3(T), lds, s, b.psi2, n, ilog2(n), b.vstat_R, d.R_min,
                           d.hR, b.r, 2, d.mp, b.kin_R, b.tw_R, d.dt, nullptr, b.flags);
    }
}

namespace {
__global__ void k_to_f32(const double2 *__restrict__ src, float2 *__restrict__ dst, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}
}  // namespace

void launch_psi1_f32(const Dims &d, const Bufs &b, hipStream_t s) {
    const size_t n = (size_t)padded(d.N) * d.nr;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b.psi1, b.psi1_f32, n);
}

}  // namespace icwf
