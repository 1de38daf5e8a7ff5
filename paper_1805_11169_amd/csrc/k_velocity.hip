// Bohmian velocities of the ICWF ansatz (Eqs. 10-11), evaluated at every
// trajectory, and the explicit-Euler trajectory update x_k+1 = x_k + dt v_k:
//     Psi_a = sum_b C_b psi1_b(r^a) psi2_b(R^a)
//     v_r^a = Im[ sum_b C_b psi2_b(R^a) d_r psi1_b(r^a) / Psi_a ] / m_r
//     v_R^a = Im[ sum_b C_b psi1_b(r^a) d_R psi2_b(R^a) / Psi_a ] / m_R
// CWF values off the grid are band-limited interpolants: f(x) = sum_i f_i S(x - x_i)
// with the periodic sinc S(y) = sin(pi y/h) cos(pi y/L) / (n sin(pi y/L))
// (Trefethen, Spectral Methods in MATLAB, ch. 3; even n, Nyquist mode split
// symmetrically).
//
// 1. k_sinc: one work-group per trajectory builds S(x^a - x_i) and S'(x^a - x_i)
//    for all i.  The derivative entry of the grid point nearest x^a is set to
//    minus the sum of all others (the derivatives of the interpolant of a
//    constant vanish), which removes the cancellation of the closed form there.
// 2. k_vel_gemm: the four real x complex contractions
//        A1 = S_r psi1^T, D1 = S'_r psi1^T, A2 = S_R psi2^T, D2 = S'_R psi2^T
//    on FP64 matrix cores (v_mfma_f64_16x16x4), 64 (a) x 32 (b) tiles staged
//    through LDS, followed in registers by the b-sums with C over the tile.
// 3. k_vel_finish: sums the tile partials, forms v, updates x, raises flags,
//    and writes the per-CWF constant potential phases the propagation uses.
//    With Heun trajectories a second pass after the coefficient update
//    evaluates the field of the new state at the Euler predictor and applies
//    the trapezoid corrector x_k + dt/2 (v_k + v~).
#include "icwf_plan.hpp"
#include "icwf_expi.hpp"

namespace icwf {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mfma_f64(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void k_sinc(const double *__restrict__ pos, int Np, int n, double x_min, double h,
                       double *__restrict__ S, double *__restrict__ Sp, const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    pos = zshift(pos, zo_);
    S = zshift(S, zo_);
    Sp = zshift(Sp, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    __shared__ double red[256];
    const int a = blockIdx.x;
    const int tid = threadIdx.x;
    const double u = (pos[a] - x_min) / h;          // position in grid units
    long long nr = (long long)floor(u + 0.5);
    const int near = (int)(((nr % n) + n) % n);
    double sp, cp;
    sincospi(u, &sp, &cp);
    const double inv_n = 1.0 / n;
    const double dscale = kPi / (n * h);
    double dsum = 0.0;
    double *Srow = S + (size_t)a * n;
    double *Dprow = Sp + (size_t)a * n;
    for (int i = tid; i < n; i += blockDim.x) {
        const double sgn = (i & 1) ? -1.0 : 1.0;
        const double sa = sgn * sp, ca = sgn * cp;   // sin, cos of pi (u - i)
        double d = u - (double)i;                    // exact
        if (i == near) d -= n * rint(d * inv_n);     // periodic image in [-1/2, 1/2]
        double sb, cb;
        sincospi(d * inv_n, &sb, &cb);
        double val, der = 0.0;
        if (i == near && fabs(d) < 1e-7) {
            const double a2 = kPi * kPi * d * d;
            val = 1.0 - a2 * (1.0 / 6.0 + inv_n * inv_n / 3.0);
        } else {
            val = sa * cb / (n * sb);
        }
        if (i != near) {
            der = dscale * (ca * cb / sb - sa * inv_n / (sb * sb));
            dsum += der;
        }
        Srow[i] = val;
        Dprow[i] = der;
    }
    red[tid] = dsum;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) Dprow[near] = -red[0];
}

// Work-group of 4 waves per 64 (a) x 32 (b) tile, wave w on the rows
// a0 + 16 w .. + 15 against all 32 columns (two MFMA fragments, rows = a,
// columns = b, k the grid index).  Lane l supplies A = table[a][k] and
// B = psi[b][k] with a, b = l % 16 of the fragment and k = l / 16 of the k
// step.  The 64 table rows (S and S') and the 32 psi rows of a 16-wide k
// chunk are staged in LDS by coalesced loads (two buffers: the loads of chunk
// c + 1 are in flight while the matrix cores work on chunk c); species r's
// chunks come first, then species R's, into their own accumulators.  The
// epilogue forms the three products with C_b and sums them over the tile's
// 32 columns (registers, then 16-lane shuffles).
constexpr int kVA = 64, kVB = 32, kVKC = 16, kVLD = kVKC + 1;

struct VelStage {
    double S[2][kVA][kVLD];
    double D[2][kVA][kVLD];
    double2 P[2][kVB][kVLD];
};

// acc[0..3][g] += (S, S') x (Re, Im) psi over the k range of one species
__device__ __forceinline__ void vel_species(const double *__restrict__ Sg, const double *__restrict__ Dg,
                                   const double2 *__restrict__ Pg, int K, int a0, int b0, VelStage &st,
                                   dbl4 (&acc)[4][2]) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int row = lane & 15, quarter = lane >> 4;
    // staging: table element e = t + 256 m (m < 4) is row e / 16, k e % 16;
    // psi element e = t + 256 m (m < 2) likewise
    const int srow = t >> 4, sk = t & 15;
    const double *sp = Sg + (size_t)(a0 + srow) * K + sk;
    const double *dp = Dg + (size_t)(a0 + srow) * K + sk;
    const double2 *pp = Pg + (size_t)(b0 + srow) * K + sk;
    const size_t rs = (size_t)16 * K;
    // staged values held as plain doubles (an array of double2 would be
    // placed in scratch memory)
    double rsv[4], rdv[4], rpx[2], rpy[2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        rsv[m] = sp[m * rs];
        rdv[m] = dp[m * rs];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double2 p = pp[m * rs];
        rpx[m] = p.x;
        rpy[m] = p.y;
    }
    __syncthreads();                         // the previous user of the buffers is done
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        st.S[0][srow + 16 * m][sk] = rsv[m];
        st.D[0][srow + 16 * m][sk] = rdv[m];
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) st.P[0][srow + 16 * m][sk] = make_double2(rpx[m], rpy[m]);
    __syncthreads();
    const int nch = K / kVKC;
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) {
            const int k0 = (ch + 1) * kVKC;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                rsv[m] = sp[m * rs + k0];
                rdv[m] = dp[m * rs + k0];
            }
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const double2 p = pp[m * rs + k0];
                rpx[m] = p.x;
                rpy[m] = p.y;
            }
        }
#pragma unroll
        for (int s4 = 0; s4 < kVKC / 4; ++s4) {
            const int kk = 4 * s4 + quarter;
            const double sv = st.S[buf][16 * wave + row][kk];
            const double dv = st.D[buf][16 * wave + row][kk];
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const double2 pv = st.P[buf][16 * g + row][kk];
                acc[0][g] = mfma_f64(sv, pv.x, acc[0][g]);
                acc[1][g] = mfma_f64(sv, pv.y, acc[1][g]);
                acc[2][g] = mfma_f64(dv, pv.x, acc[2][g]);
                acc[3][g] = mfma_f64(dv, pv.y, acc[3][g]);
            }
        }
        if (more) {
            const int nb = buf ^ 1;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                st.S[nb][srow + 16 * m][sk] = rsv[m];
                st.D[nb][srow + 16 * m][sk] = rdv[m];
            }
#pragma unroll
            for (int m = 0; m < 2; ++m) st.P[nb][srow + 16 * m][sk] = make_double2(rpx[m], rpy[m]);
        }
        __syncthreads();
    }
}

template <bool BATCHED>
__global__ void __launch_bounds__(256) k_vel_gemm(const double *__restrict__ Sr, const double *__restrict__ Dr,
                                                  const double2 *__restrict__ psi1, int nr,
                                                  const double *__restrict__ SR, const double *__restrict__ DR,
                                                  const double2 *__restrict__ psi2, int nR,
                                                  const double2 *__restrict__ C, int Np,
                                                  double2 *__restrict__ part, const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = BATCHED ? batch_offset(zoff) : 0;
    Sr = zshift(Sr, zo_);
    Dr = zshift(Dr, zo_);
    psi1 = zshift(psi1, zo_);
    SR = zshift(SR, zo_);
    DR = zshift(DR, zo_);
    psi2 = zshift(psi2, zo_);
    C = zshift(C, zo_);
    part = zshift(part, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    __shared__ VelStage st;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15;
    const int a0 = blockIdx.x * kVA, b0 = blockIdx.y * kVB;
    // [0] S psi.re, [1] S psi.im, [2] S' psi.re, [3] S' psi.im per column fragment
    dbl4 x1[4][2], x2[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            x1[i][g] = dbl4{0, 0, 0, 0};
            x2[i][g] = dbl4{0, 0, 0, 0};
        }
    vel_species(Sr, Dr, psi1, nr, a0, b0, st, x1);
    vel_species(SR, DR, psi2, nR, a0, b0, st, x2);
    // epilogue: this lane holds columns b = b0 + 16 g + row, rows
    // a = a0 + 16 wave + mfma_row_f64(lane, v)
    const double2 cb0 = C[b0 + row], cb1 = C[b0 + 16 + row];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double2 pPsi = make_double2(0.0, 0.0), pr = pPsi, pR = pPsi;
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const double2 A1 = make_double2(x1[0][g][v], x1[1][g][v]);
            const double2 D1 = make_double2(x1[2][g][v], x1[3][g][v]);
            const double2 A2 = make_double2(x2[0][g][v], x2[1][g][v]);
            const double2 D2 = make_double2(x2[2][g][v], x2[3][g][v]);
            const double2 cb = g ? cb1 : cb0;
            const double2 cA2 = cmul(cb, A2);
            pPsi = cadd(pPsi, cmul(cA2, A1));
            pr = cadd(pr, cmul(cA2, D1));
            pR = cadd(pR, cmul(cmul(cb, A1), D2));
        }
        // sum over the 16 columns held by lanes 16 quarter .. 16 quarter + 15
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            pPsi.x += __shfl_xor(pPsi.x, off, 16);
            pPsi.y += __shfl_xor(pPsi.y, off, 16);
            pr.x += __shfl_xor(pr.x, off, 16);
            pr.y += __shfl_xor(pr.y, off, 16);
            pR.x += __shfl_xor(pR.x, off, 16);
            pR.y += __shfl_xor(pR.y, off, 16);
        }
        if (row == 0) {
            const int a = a0 + 16 * wave + mfma_row_f64(lane, v);
            double2 *dst = part + ((size_t)blockIdx.y * Np + a) * 3;
            dst[0] = pPsi;
            dst[1] = pr;
            dst[2] = pR;
        }
    }
}

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

__global__ void k_vel_finish(const double2 *__restrict__ part, int N, int Np, double m_r, double m_R, double dt,
                             double *__restrict__ r, double *__restrict__ R, double *__restrict__ r_new,
                             double *__restrict__ R_new, double *__restrict__ v_r, double *__restrict__ v_R,
                             double2 *__restrict__ psi_at, double r_lo, double r_hi, double R_lo, double R_hi,
                             ModelParams mp, double2 *__restrict__ cphase, int mode, int32_t *__restrict__ flags,
                             unsigned long long *__restrict__ min_bits, const long long *__restrict__ zoff, const ModelParams *__restrict__ mpd) {
    const long long zo_ = batch_offset(zoff);
    part = zshift(part, zo_);
    r = zshift(r, zo_);
    R = zshift(R, zo_);
    r_new = zshift(r_new, zo_);
    R_new = zshift(R_new, zo_);
    v_r = zshift(v_r, zo_);
    v_R = zshift(v_R, zo_);
    psi_at = zshift(psi_at, zo_);
    cphase = zshift(cphase, zo_);
    flags = zshift(flags, zo_);
    min_bits = zshift(min_bits, zo_);
    if (zoff) mp = *zshift(mpd, zo_);

    if (flags[kFlagHalt]) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    // the phases e^{-i V dt/2} of the one-coordinate potential part that is
    // constant on the grid of each CWF conditioned on this trajectory (V_2 at
    // R^a for the electronic CWF, V_1 at r^a for the nuclear one), at the
    // positions the propagation of this step conditions on
    if (mode == kVelocityEuler) {
        cphase[a] = expi(-0.5 * dt * model_v2(mp, R[a]));
        cphase[Np + a] = expi(-0.5 * dt * model_v1(mp, r[a]));
    }
    const int ntile = Np / kVB;
    double2 ps = make_double2(0, 0), nr = make_double2(0, 0), nR = make_double2(0, 0);
    for (int t = 0; t < ntile; ++t) {
        const double2 *src = part + ((size_t)t * Np + a) * 3;
        ps = cadd(ps, src[0]);
        nr = cadd(nr, src[1]);
        nR = cadd(nR, src[2]);
    }
    const double mag2 = ps.x * ps.x + ps.y * ps.y;
    const double mag = sqrt(mag2);
    psi_at[a] = ps;
    atomicMin(min_bits, dbits(mag));
    if (!(mag >= 1e-300)) {
        atomicOr(&flags[kFlagNode], 1);
        atomicOr(&flags[kFlagHalt], 1);
        v_r[a] = 0.0;
        v_R[a] = 0.0;
        return;
    }
    // Im(n / Psi) = (n.y Psi.x - n.x Psi.y) / |Psi|^2
    const double vr = (nr.y * ps.x - nr.x * ps.y) / mag2 / m_r;
    const double vR = (nR.y * ps.x - nR.x * ps.y) / mag2 / m_R;
    if (mode == kVelocityHeun) {
        // trapezoid corrector: the first pass's v (at x_k) and this field at the predictor
        const double xr = r[a] + 0.5 * dt * (v_r[a] + vr), xR = R[a] + 0.5 * dt * (v_R[a] + vR);
        r[a] = xr;
        R[a] = xR;
        r_new[a] = xr;
        R_new[a] = xR;
        if (!isfinite(xr) || !isfinite(xR)) {
            atomicOr(&flags[kFlagNonfinite], 1);
            atomicOr(&flags[kFlagHalt], 1);
        }
        if (xr < r_lo || xr >= r_hi || xR < R_lo || xR >= R_hi) atomicAdd(&flags[kFlagOut], 1);
        return;
    }
    v_r[a] = vr;
    v_R[a] = vR;
    if (mode == kVelocityEuler) {
        const double xr = r[a] + dt * vr, xR = R[a] + dt * vR;
        r_new[a] = xr;
        R_new[a] = xR;
        if (!isfinite(xr) || !isfinite(xR)) {
            atomicOr(&flags[kFlagNonfinite], 1);
            atomicOr(&flags[kFlagHalt], 1);
        }
        if (xr < r_lo || xr >= r_hi || xR < R_lo || xR >= R_hi) atomicAdd(&flags[kFlagOut], 1);
    }
}

__global__ void k_vel_reset(int32_t *flags, unsigned long long *min_bits, int keep_min, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    flags = zshift(flags, zo_);
    min_bits = zshift(min_bits, zo_);

    if (threadIdx.x == 0) {
        flags[kFlagOut] = 0;
        if (!keep_min) *min_bits = 0x7ff0000000000000ULL;   // +inf
    }
}

}  // namespace

void launch_velocity(const Dims &d, const Bufs &b, VelocityMode mode, hipStream_t s) {
    const int Np = padded(d.N);
    // the corrector evaluates the field at the predictor positions
    const double *pr = mode == kVelocityHeun ? b.r_new : b.r;
    const double *pR = mode == kVelocityHeun ? b.R_new : b.R;
    const int B = d.batch;
    hipLaunchKernelGGL(k_sinc, dim3(Np, 1, B), dim3(256), 0, s, pr, Np, d.nr, d.r_min, d.hr, b.sinc_r, b.dsinc_r,
                       b.flags, d.zoff);
    hipLaunchKernelGGL(k_sinc, dim3(Np, 1, B), dim3(256), 0, s, pR, Np, d.nR, d.R_min, d.hR, b.sinc_R, b.dsinc_R,
                       b.flags, d.zoff);
    hipLaunchKernelGGL(d.zoff ? k_vel_gemm<true> : k_vel_gemm<false>, dim3(Np / kVA, Np / kVB, B), dim3(256), 0, s, b.sinc_r, b.dsinc_r, b.psi1, d.nr,
                       b.sinc_R, b.dsinc_R, b.psi2, d.nR, b.C, Np, b.vpart, b.flags, d.zoff);
    unsigned long long *min_bits = reinterpret_cast<unsigned long long *>(b.scal);
    // min |Psi| over the step's evaluations: the corrector keeps the first pass's minimum
    hipLaunchKernelGGL(k_vel_reset, dim3(1, 1, B), dim3(64), 0, s, b.flags, min_bits, mode == kVelocityHeun ? 1 : 0,
                       d.zoff);
    const double r_hi = d.r_min + d.hr * d.nr, R_hi = d.R_min + d.hR * d.nR;
    hipLaunchKernelGGL(k_vel_finish, dim3((d.N + 255) / 256, 1, B), dim3(256), 0, s, b.vpart, d.N, Np, d.m_r, d.m_R,
                       d.dt, b.r, b.R, b.r_new, b.R_new, b.v_r, b.v_R, b.psi_at, d.r_min, r_hi, d.R_min, R_hi, d.mp,
                       b.cphase, (int)mode, b.flags, min_bits, d.zoff, d.mpd);
}

}  // namespace icwf
