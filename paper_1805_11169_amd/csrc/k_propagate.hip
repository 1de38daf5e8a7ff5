// Hermitian-CWF propagation (Eqs. 5-6 with the eta potentials reduced to a
// dropped phase): every conditional wavefunction takes one Strang
// split-operator step under its own conditioned potential, the conditioning
// coordinate frozen at the step's start:
//     psi <- e^{-i V dt/2} IFFT[ e^{-i k^2 dt/2m} FFT( e^{-i V dt/2} psi ) ],
//     V_1^a(r_i) = W(r_i, R^a),   V_2^a(R_j) = W(r^a, R_j).
//
// One work-group per CWF (several for small grids).  Thread t of a CWF holds
// the 8 points t + m n/8, m = 0..7: that is the set the first pass of a
// Stockham FFT reads and the set its last pass writes, so the potential phase
// and the first forward pass, the last forward pass, the kinetic phase and the
// first inverse pass, and the last inverse pass and the store all run in
// registers.  The passes between them go through two LDS buffers (radix 8, with one radix
// 2 or 4 pass first when log2 n is not a multiple of 3; twiddles from a
// table).  The CWF is read once from HBM and written once, both coalesced.
// The potential phase is evaluated once per point (one erf, one sincos) and
// kept in registers for both half steps.  The inverse FFT is the forward one
// applied to the conjugate.  Bound: HBM (2 x 16 bytes per grid point per step).
#include "icwf_plan.hpp"

namespace icwf {

namespace {

constexpr int kPts = 8;   // points per thread

// LDS position of FFT element i: one pad slot after every 8 elements.  The
// early Stockham passes write with strides 8 and 64 (element 8 t + r, and
// 64 u + k + 8 r); padded, every 16 consecutive lanes hit 16 different
// 16-byte bank groups instead of a handful.
__device__ inline int lp(int i) { return i + (i >> 3); }

__device__ inline void dft2(double2 &a, double2 &b) {
    const double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ inline void dft4(double2 &a0, double2 &a1, double2 &a2, double2 &a3) {
    double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = make_double2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
    a3 = make_double2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
}

// X[m] = sum_r u[r] W^(r m), W = exp(-2 pi i / 8): the 4-point transforms of
// the even and odd samples, combined with W^m = 1, (1 - i)/sqrt 2, -i,
// -(1 + i)/sqrt 2.
__device__ inline void dft8(double2 (&u)[8]) {
    constexpr double kS = 0.70710678118654752440;
    double2 e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6];
    double2 o0 = u[1], o1 = u[3], o2 = u[5], o3 = u[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const double2 w1 = make_double2(kS * (o1.x + o1.y), kS * (o1.y - o1.x));    // o1 (1 - i)/sqrt 2
    const double2 w2 = make_double2(o2.y, -o2.x);                               // -i o2
    const double2 w3 = make_double2(kS * (o3.y - o3.x), -kS * (o3.x + o3.y));   // -o3 (1 + i)/sqrt 2
    u[0] = cadd(e0, o0);
    u[4] = csub(e0, o0);
    u[1] = cadd(e1, w1);
    u[5] = csub(e1, w1);
    u[2] = cadd(e2, w2);
    u[6] = csub(e2, w2);
    u[3] = cadd(e3, w3);
    u[7] = csub(e3, w3);
}

// One Stockham pass of radix R, Ns = size of the sub-transforms already done.
// The thread's 8 values are 8/R butterflies; butterfly b (index
// j = t + b n/8 among the n/R of the pass) takes v[b + r 8/R], r = 0..R-1,
// read from src[j + r n/R], twiddled by exp(-2 pi i r k / (Ns R)) with
// k = j mod Ns, and its outputs go to dst[(j - k) R + k + r Ns].  The first
// pass takes its inputs from registers and the last keeps its outputs there;
// on both ends v[m] is the point t + m n/8.  src and dst are different LDS
// buffers, so one barrier per pass (after the writes) orders everything.
template <int R>
__device__ inline void fft_pass(double2 (&v)[kPts], const double2 *src, double2 *dst, int n, int Ns, int t,
                                const double2 *__restrict__ tw, bool first, bool last) {
    constexpr int S = kPts / R;
    const int q = n / kPts;
    const int nR = n / R;
    if (!first) {
#pragma unroll
        for (int b = 0; b < S; ++b)
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + r * S] = src[lp(t + b * q + r * nR)];
    }
    if (Ns > 1) {
        const int st = n / (Ns * R);
#pragma unroll
        for (int b = 0; b < S; ++b) {
            const int k = (t + b * q) & (Ns - 1);
            // w^r from one table entry w = exp(-2 pi i k / (Ns R)) by products
            // (a few ulp, far below the FFT's own rounding): one load instead
            // of R - 1 in flight per butterfly
            const double2 w = tw[(k * st) & (n - 1)];
            double2 wr = w;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                v[b + r * S] = cmul(v[b + r * S], wr);
                if (r + 1 < R) wr = cmul(wr, w);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < S; ++b) {
        if (R == 8) {
            double2 u[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) u[r] = v[b + r * S];
            dft8(u);
#pragma unroll
            for (int r = 0; r < 8; ++r) v[b + r * S] = u[r];
        } else if (R == 4) {
            dft4(v[b], v[b + S], v[b + 2 * S], v[b + 3 * S]);
        } else {
            dft2(v[b], v[b + S]);
        }
    }
    if (!last) {
#pragma unroll
        for (int b = 0; b < S; ++b) {
            const int j = t + b * q, k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) dst[lp((j - k) * R + k + r * Ns)] = v[b + r * S];
        }
        __syncthreads();
    }
}

// Forward DFT (unnormalised) of the CWF held as v[m] = x[t + m n/8]; returns
// X[t + m n/8] in v[m].  sh holds two buffers of stride ld; par is the buffer
// the next pass writes, kept across calls so that the first pass of one
// transform never writes the buffer the last pass of the previous one reads.
__device__ inline void fft8(double2 (&v)[kPts], double2 *sh, int ld, int &par, int n, int log2n, int t,
                            const double2 *__restrict__ tw) {
    const int rem = log2n % 3;
    const int npass = (log2n + 2) / 3;
    int Ns = 1, pass = 0;
    if (rem == 1) {
        fft_pass<2>(v, sh + (par ^ 1) * ld, sh + par * ld, n, Ns, t, tw, true, npass == 1);
        par ^= 1;
        Ns = 2;
        pass = 1;
    } else if (rem == 2) {
        fft_pass<4>(v, sh + (par ^ 1) * ld, sh + par * ld, n, Ns, t, tw, true, npass == 1);
        par ^= 1;
        Ns = 4;
        pass = 1;
    }
    for (; Ns < n; Ns *= 8, ++pass) {
        const bool last = pass == npass - 1;
        fft_pass<8>(v, sh + (par ^ 1) * ld, sh + par * ld, n, Ns, t, tw, pass == 0, last);
        if (!last) par ^= 1;
    }
}

// blockDim.x = max(64, n/8) threads: n/8 per CWF, blockDim.x / (n/8) CWFs.
__global__ void __launch_bounds__(512) k_propagate(double2 *__restrict__ psi, int n, int log2n,
                                                   const double *__restrict__ vstat, double x_min, double h,
                                                   const double *__restrict__ cond, int species, ModelParams mp,
                                                   const double2 *__restrict__ kin,
                                                   const double2 *__restrict__ tw, double dt,
                                                   float2 *__restrict__ psi_f32,
                                                   const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    extern __shared__ double2 sh_all[];
    const int q = n / kPts;
    const int cpb = blockDim.x / q;
    const int lc = threadIdx.x / q, t = threadIdx.x - lc * q;
    const int cw = blockIdx.x * cpb + lc;
    const int ld = n + n / 8;                // one padded buffer; two per CWF
    double2 *sh = sh_all + lc * 2 * ld;
    int par = 0;
    double2 *p = psi + (size_t)cw * n;
    const double c = cond[cw];
    // part of the conditioned potential that is constant on this CWF's grid
    const double vconst = (species == 1) ? model_v2(mp, c) : model_v1(mp, c);

    double2 ph[kPts], v[kPts];
    // the CWF's loads first: they are in flight while the phases (which do not
    // depend on them) are evaluated
#pragma unroll
    for (int m = 0; m < kPts; ++m) v[m] = p[t + m * q];
#pragma unroll
    for (int m = 0; m < kPts; ++m) {
        const int i = t + m * q;
        const double x = x_min + i * h;
        const double V = vstat[i] + vconst + ((species == 1) ? model_wc(mp, x, c) : model_wc(mp, c, x));
        double s, co;
        sincos(-0.5 * dt * V, &s, &co);
        ph[m] = make_double2(co, s);
    }
#pragma unroll
    for (int m = 0; m < kPts; ++m) v[m] = cmul(ph[m], v[m]);
    fft8(v, sh, ld, par, n, log2n, t, tw);
#pragma unroll
    for (int m = 0; m < kPts; ++m) v[m] = cconj(cmul(kin[t + m * q], v[m]));
    fft8(v, sh, ld, par, n, log2n, t, tw);
    const double inv_n = 1.0 / n;
#pragma unroll
    for (int m = 0; m < kPts; ++m) {
        const int i = t + m * q;
        const double2 o = cmul(ph[m], cscale(cconj(v[m]), inv_n));
        p[i] = o;
        // FP32 copy for the mixed form's FP32 contraction
        if (psi_f32) psi_f32[(size_t)cw * n + i] = make_float2((float)o.x, (float)o.y);
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
    const int q = n / kPts;
    const int T = q < 64 ? 64 : q;           // 64 / q CWFs per work-group below n = 512
    const int cpb = T / q;
    const int grid = padded(d.N) / cpb;      // padded rows hold zero CWFs
    const size_t lds = sizeof(double2) * (size_t)2 * (n + n / 8) * cpb;
    if (species == 1) {
        hipLaunchKernelGGL(k_propagate, dim3(grid), dim3(T), lds, s, b.psi1, n, ilog2(n), b.vstat_r, d.r_min,
                           d.hr, b.R, 1, d.mp, b.kin_r, b.tw_r, d.dt, d.prec == 1 ? b.psi1_f32 : nullptr,
                           b.flags);
    } else {
        hipLaunchKernelGGL(k_propagate, dim3(grid), dim3(T), lds, s, b.psi2, n, ilog2(n), b.vstat_R, d.R_min,
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
