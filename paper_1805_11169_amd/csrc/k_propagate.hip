// Hermitian-CWF propagation (Eqs. 5-6 with the eta potentials reduced to a
// dropped phase): every conditional wavefunction takes one Strang
// split-operator step under its own conditioned potential, the conditioning
// coordinate frozen at the step's start:
//     psi <- e^{-i V dt/2} IFFT[ e^{-i k^2 dt/2m} FFT( e^{-i V dt/2} psi ) ],
//     V_1^a(r_i) = W(r_i, R^a),   V_2^a(R_j) = W(r^a, R_j).
//
// Persistent work-groups: each holds one CWF at a time (several for small
// grids) and walks the CWFs with the grid's stride, so the tables it keeps in
// LDS are loaded once per work-group and the stores of one CWF drain while the
// next one is read and its phases are evaluated.  Thread t of a CWF holds the
// 8 points t + m n/8, m = 0..7: that is the set the first pass of a Stockham
// FFT reads and the set its last pass writes, so the potential phase and the
// first forward pass, the last forward pass, the kinetic phase and the first
// inverse pass, and the last inverse pass and the store all run in registers.
// The passes between them go through two LDS buffers (radix 8, with one
// radix 2 or 4 pass first when log2 n is not a multiple of 3; twiddles from an
// LDS table); n = 4096 uses a four-step 64 x 64 transform through one buffer
// instead (below).  The CWF is read once from HBM and written once, both
// coalesced.  The potential phase is evaluated once per point and kept in
// registers for both half steps, as the product of a table of the
// one-coordinate part's phase, the constant part's phase (per CWF, written by
// the velocity kernel), and the coupling's (from a piecewise-polynomial erf
// table, e^{i theta} by a Taylor series, reduced when needed).  The inverse
// FFT is the forward one applied to the conjugate.
#include <cmath>

#include "icwf_plan.hpp"
#include "icwf_expi.hpp"

#include "erf_table.inc"

namespace icwf {

namespace {

constexpr int kPts = 8;   // points per thread
// the erf(z)/z table in LDS, in 16-byte slots
constexpr int kErfTableSlots = (kErfPieces * kErfTerms * 8 + 15) / 16;
// the 64th roots of unity w64^(a b), a, b < 8, of the four-step transform
constexpr int kW64Slots = 64;

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
                                const double2 *tw, bool first, bool last) {
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
            // (a few ulp, far below the FFT's own rounding); k st < n / 8, so
            // the table holds exp(-2 pi i j / n) for j < n / 8 only
            const double2 w = tw[k * st];
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
// n = 2^LOG2N is a compile-time constant, so the passes unroll and every LDS
// index becomes a per-thread base plus an immediate offset.
template <int LOG2N>
__device__ inline void fft8(double2 (&v)[kPts], double2 *sh, int ld, int &par, int t, const double2 *tw) {
    constexpr int n = 1 << LOG2N;
    constexpr int rem = LOG2N % 3;
    constexpr int npass = (LOG2N + 2) / 3;
    constexpr int first8 = rem ? 1 : 0;      // index of the first radix-8 pass
    if constexpr (rem == 1) {
        fft_pass<2>(v, sh + (par ^ 1) * ld, sh + par * ld, n, 1, t, tw, true, npass == 1);
        par ^= 1;
    } else if constexpr (rem == 2) {
        fft_pass<4>(v, sh + (par ^ 1) * ld, sh + par * ld, n, 1, t, tw, true, npass == 1);
        par ^= 1;
    }
#pragma unroll
    for (int pass = first8; pass < npass; ++pass) {
        const int Ns = (rem == 0 ? 1 : (1 << rem)) << (3 * (pass - first8));
        const bool last = pass == npass - 1;
        fft_pass<8>(v, sh + (par ^ 1) * ld, sh + par * ld, n, Ns, t, tw, pass == 0, last);
        if (!last) par ^= 1;
    }
}

// ---- n = 4096: four-step transform, one LDS buffer, four barriers per CWF ----
//
// 4096 = 64 x 64 with i = i1 + 64 i2 and k = k2 + 64 k1: a 64-point DFT over
// i2 for each i1, the twiddle w4096^(i1 k2), a 64-point DFT over i1 for each
// k2.  Each 64-point DFT is 8 x 8: an in-register radix-8 DFT, a w64 twiddle,
// an 8 x 8 exchange among 8 lanes of one wave and a second radix-8 DFT.  With
// wave w, lane l = lo + 8 hi (lo = l & 7, hi = l >> 3) and register m, the
// thread holds x[lo + 8 w + 64 hi + 512 m] on entry (i1 = lo + 8 w) and returns
// X[hi + 8 w + 64 lo + 512 m].  Only the exchange between the two halves
// crosses waves (one barrier); the 8-lane exchanges go through the wave's own
// 512-slot slice of an LDS buffer and need no barrier, LDS operations of one
// wave being executed in order.  Slot maps are XOR-swizzled so that every 16
// consecutive lanes touch 16 different 16-byte bank groups on both the write
// and the read side.
//
// The same stages in reverse order (the DFT matrix and each stage matrix being
// symmetric, up to the inverse permutations) compute the DFT from the output
// layout back to the input layout; the inverse transform is that sequence
// applied to the conjugate.  Buffer use: one 4096-slot buffer per CWF, so that
// two work-groups (sixteen waves) share a compute unit and one group's
// exchanges and barriers overlap the other's arithmetic.  Wave w's slice is
// touched by other waves only through the cross-wave writes, and the wave
// reads in the cross-wave exchange only its own slice; a barrier before each
// cross-wave write (every wave done with its slice) and the one after it
// order all accesses.

constexpr int kFourStepLog2 = 12;

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// element (lo, a, b) of the first 8 x 8 exchange (lanes (lo, a) -> (lo, b))
__device__ inline int slot_a(int lo, int a, int b) { return 64 * a + 8 * (b ^ (a & 1)) + lo; }
// element (b, p, e) of the second one (lanes (p, b) -> (e, b))
__device__ inline int slot_c(int b, int p, int e) { return 64 * b + 8 * (e ^ (b & 1)) + (p ^ e); }

// v[r] *= w64^(a r), r = 1..7, from the LDS table w64[8 a + r] of the 64th
// roots of unity w64^(a r), a, r < 8
__device__ inline void twiddle_row(double2 (&v)[kPts], const double2 *w64, int a) {
#pragma unroll
    for (int r = 1; r < kPts; ++r) v[r] = cmul(v[r], w64[8 * a + r]);
}

// v[c] *= w4096^(i1 (hi + 8 c)), c = 0..7
__device__ inline void twiddle_middle(double2 (&v)[kPts], int i1, int hi, const double2 *tw) {
    double2 t = tw[i1 * hi];
    const double2 r = tw[8 * i1];
#pragma unroll
    for (int c = 0; c < kPts; ++c) {
        v[c] = cmul(v[c], t);
        if (c + 1 < kPts) t = cmul(t, r);
    }
}

// all eight values to dest wave j = 0..7, then the eight from source waves
__device__ inline void cross_wave(double2 (&v)[kPts], double2 *B, int w, int l) {
#pragma unroll
    for (int j = 0; j < kPts; ++j) B[j * 512 + w * 64 + l] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPts; ++j) v[j] = B[w * 512 + j * 64 + l];
}

// forward, input layout -> output layout
__device__ inline void fft4096_fwd(double2 (&v)[kPts], double2 *B, int w, int l, const double2 *tw,
                                   const double2 *w64) {
    const int lo = l & 7, hi = l >> 3;
    double2 *R = B + w * 512;
    dft8(v);                                              // over i2's high part
    twiddle_row(v, w64, hi);                              // w64^(a b), a = hi
#pragma unroll
    for (int b = 0; b < kPts; ++b) R[slot_a(lo, hi, b)] = v[b];
    wave_sync();
#pragma unroll
    for (int a = 0; a < kPts; ++a) v[a] = R[slot_a(lo, a, hi)];
    dft8(v);                                              // over i2's low part
    twiddle_middle(v, lo + 8 * w, hi, tw);
    __syncthreads();                                      // every slice read by its wave
    cross_wave(v, B, w, l);
    dft8(v);                                              // over i1's high part
    twiddle_row(v, w64, lo);                              // w64^(p e), p = lo
#pragma unroll
    for (int e = 0; e < kPts; ++e) R[slot_c(hi, lo, e)] = v[e];
    wave_sync();
#pragma unroll
    for (int p = 0; p < kPts; ++p) v[p] = R[slot_c(hi, p, lo)];
    dft8(v);                                              // over i1's low part
}

// the same stages in reverse: output layout -> input layout
__device__ inline void fft4096_rev(double2 (&v)[kPts], double2 *B, int w, int l, const double2 *tw,
                                   const double2 *w64) {
    const int lo = l & 7, hi = l >> 3;
    double2 *R = B + w * 512;
    dft8(v);
#pragma unroll
    for (int p = 0; p < kPts; ++p) R[slot_c(hi, p, lo)] = v[p];
    wave_sync();
#pragma unroll
    for (int e = 0; e < kPts; ++e) v[e] = R[slot_c(hi, lo, e)];
    twiddle_row(v, w64, lo);
    dft8(v);
    __syncthreads();                                      // every slice read by its wave
    cross_wave(v, B, w, l);
    twiddle_middle(v, lo + 8 * w, hi, tw);
    dft8(v);
#pragma unroll
    for (int a = 0; a < kPts; ++a) R[slot_a(lo, a, hi)] = v[a];
    wave_sync();
#pragma unroll
    for (int b = 0; b < kPts; ++b) v[b] = R[slot_a(lo, hi, b)];
    twiddle_row(v, w64, hi);
    dft8(v);
}

// e^{i theta} for |theta| <= 0.05: the Taylor series of sin and cos to
// degrees 9 and 8, whose first dropped terms, below 0.05^10/11! = 2.5e-21
// (relative to theta) and 0.05^10/10! = 2.7e-20, are far under an ulp.
constexpr double kTinyPhase = 0.05;
__device__ inline double2 expi_tiny(double th) {
    const double u = th * th;
    double s = 1.0 / 362880.0;                    // +1/9!
    s = fma(s, u, -1.0 / 5040.0);                 // -1/7!
    s = fma(s, u, 1.0 / 120.0);                   // +1/5!
    s = fma(s, u, -1.0 / 6.0);                    // -1/3!
    double c = 1.0 / 40320.0;                     // +1/8!
    c = fma(c, u, -1.0 / 720.0);                  // -1/6!
    c = fma(c, u, 1.0 / 24.0);                    // +1/4!
    c = fma(c, u, -0.5);                          // -1/2!
    return make_double2(fma(u, c, 1.0), fma(th * u, s, th));
}

// The Shin-Metiu coupling g(d) = erf(|d|/a)/|d| at z = |d|/a: below z = 6
// from the piecewise polynomial table of erf(z)/z (read from LDS, where the
// work-group keeps it; every lane takes its own piece, no branches), above it
// 1/|d| by a reciprocal refined by two Newton steps, since erf(z) rounds to 1
// there.  inv_a = 1/a.
__device__ inline double erf_over_x_table(double d, double inv_a, const double *tab) {
    const double ax = fabs(d);
    const double z = ax * inv_a;
    double r = __builtin_amdgcn_rcp(ax);
    r = fma(fma(-ax, r, 1.0), r, r);
    r = fma(fma(-ax, r, 1.0), r, r);
    // the table only where some lane of the wave needs it (on a wide grid
    // about half of the point groups lie beyond z = 6 for every lane)
    if (__builtin_amdgcn_ballot_w64(z < 6.0) == 0) return r;
    const int j = (int)fmin(z * 4.0, (double)(kErfPieces - 1));
    const double s = z - (j + 0.5) * 0.25;
    const double *cf = tab + j * kErfTerms;
    double e = cf[kErfTerms - 1];
#pragma unroll
    for (int k = kErfTerms - 2; k >= 0; --k) e = fma(e, s, cf[k]);
    return z < 6.0 ? e * inv_a : r;
}

// Read-only data in the constant address space: with a wave-uniform index the
// loads become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) double *ConstDouble;

// x, known to be equal on all lanes, moved to SGPRs
__device__ inline double wave_uniform(double x) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// n = 2^LOG2N points; blockDim.x = max(64, n/8) threads: n/8 per CWF,
// cpb = blockDim.x / (n/8) CWFs per work-group; work-group g takes the CWF
// groups g, g + G, ... of the ngroups = Np / cpb (G = gridDim.x).  LDS: the
// n/8 twiddles, the erf(z)/z table, the w64^(a b) table, then per CWF two
// (padded) buffers, one at n = 4096.  At n = 4096 the kernel is held to 128
// VGPRs (four waves per SIMD), so that two work-groups fit a compute unit;
// for that the per-CWF constant phase comes precomputed (cph) rather than
// from the model's erf, whose constants would stay in registers across the
// loop, and every global access is a uniform base plus a 32-bit lane offset.
template <int LOG2N, bool BATCHED>
__global__ void __launch_bounds__(512, LOG2N == kFourStepLog2 ? 4 : 1)
    k_propagate(double2 *__restrict__ psi, int ngroups, const double2 *__restrict__ vphase, double x_min, double h,
                const double *__restrict__ cond, const double2 *__restrict__ cph, int species, ModelParams mp,
                const double2 *__restrict__ kin, const double2 *__restrict__ tw, double dt, int tiny,
                float2 *__restrict__ psi_f32, const int32_t *__restrict__ flags, const long long *__restrict__ zoff, const ModelParams *__restrict__ mpd) {
    const long long zo_ = BATCHED ? batch_offset(zoff) : 0;
    psi = zshift(psi, zo_);
    vphase = zshift(vphase, zo_);
    cond = zshift(cond, zo_);
    cph = zshift(cph, zo_);
    kin = zshift(kin, zo_);
    tw = zshift(tw, zo_);
    psi_f32 = zshift(psi_f32, zo_);
    flags = zshift(flags, zo_);
    if (BATCHED) mp = *zshift(mpd, zo_);

    if (flags[kFlagHalt]) return;
    extern __shared__ double2 sh_all[];
    constexpr int n = 1 << LOG2N;
    constexpr int q = n / kPts;
    constexpr int cpb = q < 64 ? 64 / q : 1;
    constexpr bool four_step = LOG2N == kFourStepLog2;
    constexpr int ld = four_step ? n : n + n / 8;   // one (padded) buffer
    constexpr int nbuf = four_step ? 1 : 2;         // buffers per CWF
    // points whose potential phases are evaluated together: at 128 VGPRs one
    // at a time, else two (all eight in flight at once need more registers
    // than the wave has)
    constexpr int group = four_step ? 1 : 2;
    const int lc = threadIdx.x / q, t0 = threadIdx.x - lc * q;
    double2 *stw = sh_all;
    double *serf = reinterpret_cast<double *>(sh_all + q);
    double2 *sw64 = sh_all + q + kErfTableSlots;
    double2 *sh = sh_all + q + kErfTableSlots + kW64Slots + lc * nbuf * ld;
    for (int j = threadIdx.x; j < q; j += blockDim.x) stw[j] = tw[j];
    if constexpr (LOG2N == kFourStepLog2)
        for (int j = threadIdx.x; j < kW64Slots; j += blockDim.x) sw64[j] = tw[64 * (j >> 3) * (j & 7)];
    for (int j = threadIdx.x; j < kErfPieces * kErfTerms; j += blockDim.x) serf[j] = (&kErfOverZ[0][0])[j];
    int par = 0;
    // this thread's points: x index xi + m q, FFT-order k index ki + m q
    int xi0 = t0, ki0 = t0;
    if constexpr (four_step) {
        const int w = t0 >> 6, lo = t0 & 7, hi = (t0 >> 3) & 7;
        xi0 = lo + 8 * w + 64 * hi;
        ki0 = hi + 8 * w + 64 * lo;
    }
    // the conditioning coordinate and the constant phase are read one CWF
    // ahead: the phases of a CWF cannot start before they arrive.  With one
    // CWF per work-group they are uniform: scalar loads, held in SGPRs.
    double c_next = 0.0;
    double2 pc_next = make_double2(0.0, 0.0);
    auto fetch = [&](int gn) {
        if constexpr (cpb == 1) {
            c_next = ((ConstDouble)cond)[gn];
            const ConstDouble pp = (ConstDouble)cph;
            pc_next = make_double2(pp[2 * gn], pp[2 * gn + 1]);
        } else {
            c_next = cond[gn * cpb + lc];
            pc_next = cph[gn * cpb + lc];
        }
    };
    if (blockIdx.x < (unsigned)ngroups) fetch(blockIdx.x);
    const double inv_a = wave_uniform(1.0 / mp.p[1]);   // Shin-Metiu: 1/R_f
    __syncthreads();                         // tables in place
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        // the thread index, opaque to the compiler within each iteration:
        // otherwise the loads and addresses that do not change from one CWF
        // to the next are hoisted out of the loop and held in registers
        // across it, which spills
        int t = t0, xi = xi0, ki = ki0;
        asm volatile("" : "+v"(t), "+v"(xi), "+v"(ki));
        const unsigned ux = (unsigned)xi, uk = (unsigned)ki;
        const int cw = g * cpb + lc;
        double2 *p = psi + (size_t)cw * n;
        const double c = c_next;
        const double2 pc = pc_next;          // e^{-i V_c dt/2}, V_c the part of the potential constant on the grid
        if (g + (int)gridDim.x < ngroups) fetch(g + gridDim.x);
        double2 v[kPts];
#pragma unroll
        for (int m = 0; m < kPts; ++m) v[m] = (p + m * q)[ux];
        // e^{-i V dt/2} = e^{-i V_s(x) dt/2} (table) x e^{-i V_c dt/2} x
        // e^{-i W_c(x) dt/2} (the coupling, evaluated per point)
        double2 ph[kPts];
        if (mp.kind == 1) {                  // Shin-Metiu: W_c = -g(r - R; R_f), 0 <= g <= 2/(sqrt(pi) R_f)
            if (tiny) {                      // dt/(sqrt(pi) R_f) <= kTinyPhase
#pragma unroll
                for (int m = 0; m < kPts; ++m) {
                    const double x = x_min + (xi + m * q) * h;
                    const double2 e = expi_tiny(0.5 * dt * erf_over_x_table(x - c, inv_a, serf));
                    ph[m] = cmul(cmul((vphase + m * q)[ux], pc), e);
                    if (m % group == group - 1) __builtin_amdgcn_sched_barrier(0);
                }
            } else {
#pragma unroll
                for (int m = 0; m < kPts; ++m) {
                    const double x = x_min + (xi + m * q) * h;
                    const double2 e = expi(0.5 * dt * erf_over_x_table(x - c, inv_a, serf));
                    ph[m] = cmul(cmul((vphase + m * q)[ux], pc), e);
                    if (m % group == group - 1) __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < kPts; ++m) {
                const double x = x_min + (xi + m * q) * h;
                const double wcv = (species == 1) ? model_wc(mp, x, c) : model_wc(mp, c, x);
                ph[m] = cmul(cmul((vphase + m * q)[ux], pc), expi(-0.5 * dt * wcv));
                if (m % group == group - 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int m = 0; m < kPts; ++m) v[m] = cmul(ph[m], v[m]);
        // the kinetic phases: ahead of the forward transform where registers
        // allow, after it at 128 VGPRs
        double2 kv[kPts];
        if constexpr (!four_step) {
#pragma unroll
            for (int m = 0; m < kPts; ++m) kv[m] = (kin + m * q)[uk];
            fft8<LOG2N>(v, sh, ld, par, t, stw);
        } else {
            fft4096_fwd(v, sh, t >> 6, t & 63, stw, sw64);
#pragma unroll
            for (int m = 0; m < kPts; ++m) kv[m] = (kin + m * q)[uk];
        }
#pragma unroll
        for (int m = 0; m < kPts; ++m) v[m] = cconj(cmul(kv[m], v[m]));
        if constexpr (four_step) fft4096_rev(v, sh, t >> 6, t & 63, stw, sw64);
        else fft8<LOG2N>(v, sh, ld, par, t, stw);
        float2 *pf = psi_f32 ? psi_f32 + (size_t)cw * n : nullptr;
#pragma unroll
        for (int m = 0; m < kPts; ++m) {
            const double2 o = cmul(ph[m], cconj(v[m]));   // the 1/n of the inverse is in the kinetic table
            (p + m * q)[ux] = o;
            // FP32 copy for the mixed form's FP32 contraction
            if (pf) (pf + m * q)[ux] = make_float2((float)o.x, (float)o.y);
        }
    }
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

namespace {
int threads_for(int n) {
    const int q = n / kPts;
    return q < 64 ? 64 : q;                  // 64 / q CWFs per work-group below n = 512
}
size_t lds_for(int n) {
    const int q = n / kPts;
    const int cpb = threads_for(n) / q;
    const size_t ld = ilog2(n) == kFourStepLog2 ? n : n + n / 8;
    const size_t nbuf = ilog2(n) == kFourStepLog2 ? 1 : 2;
    return sizeof(double2) * ((size_t)q + kErfTableSlots + kW64Slots + nbuf * ld * cpb);
}
}  // namespace

namespace {
// The instantiation for n = 2^l, 32 <= n <= 4096.
using PropKernel = void (*)(double2 *, int, const double2 *, double, double, const double *, const double2 *, int,
                            ModelParams, const double2 *, const double2 *, double, int, float2 *, const int32_t *,
                            const long long *, const ModelParams *);
template <bool B>
PropKernel kernel_for_t(int n) {
    switch (ilog2(n)) {
    case 5: return k_propagate<5, B>;
    case 6: return k_propagate<6, B>;
    case 7: return k_propagate<7, B>;
    case 8: return k_propagate<8, B>;
    case 9: return k_propagate<9, B>;
    case 10: return k_propagate<10, B>;
    case 11: return k_propagate<11, B>;
    case 12: return k_propagate<12, B>;
    default: return nullptr;
    }
}
// batched: the instantiation with the per-simulation offsets (launches of
// one simulation keep the kernel without them)
PropKernel kernel_for(int n, bool batched = false) { return batched ? kernel_for_t<true>(n) : kernel_for_t<false>(n); }
}  // namespace

int propagate_grid(int n, int N, int ncu) {
    const int T = threads_for(n);
    const int ngroups = padded(N) / (T / (n / kPts));
    int per_cu = 0;
    const PropKernel k = kernel_for(n);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, T, lds_for(n)) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const long long full = (long long)per_cu * (ncu > 0 ? ncu : 1);
    return (int)(ngroups < full ? ngroups : full);
}

bool propagate_tiny_phase(const Dims &d) {
    return d.mp.kind == 1 && 0.5 * std::fabs(d.dt) * 2.0 / (std::sqrt(M_PI) * d.mp.p[1]) <= kTinyPhase;
}

void launch_propagate(const Dims &d, const Bufs &b, int species, hipStream_t s) {
    if (d.propagator == 1) {
        launch_propagate_cn(d, b, species, s);
        return;
    }
    const int n = species == 1 ? d.nr : d.nR;
    const int T = threads_for(n);
    const int ngroups = padded(d.N) / (T / (n / kPts));   // padded rows hold zero CWFs
    const int grid = d.prop_grid[species - 1];
    const size_t lds = lds_for(n);
    const PropKernel k = kernel_for(n, d.zoff != nullptr);   // n validated at creation: a power of two in [32, 4096]
    // the Shin-Metiu coupling phase stays within the short series' range
    const int tiny = propagate_tiny_phase(d) ? 1 : 0;
    if (species == 1) {
        hipLaunchKernelGGL(k, dim3(grid, 1, d.batch), dim3(T), lds, s, b.psi1, ngroups, b.vphase_r, d.r_min, d.hr, b.R,
                           b.cphase, 1, d.mp, b.kin_r, b.tw_r, d.dt, tiny,
                           d.prec == 1 && d.fp32_residual ? b.psi1_f32 : nullptr, b.flags, d.zoff, d.mpd);
    } else {
        hipLaunchKernelGGL(k, dim3(grid, 1, d.batch), dim3(T), lds, s, b.psi2, ngroups, b.vphase_R, d.R_min, d.hR, b.r,
                           b.cphase + padded(d.N), 2, d.mp, b.kin_R, b.tw_R, d.dt, tiny, nullptr, b.flags, d.zoff, d.mpd);
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
