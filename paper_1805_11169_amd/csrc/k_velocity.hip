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
//    on FP64 matrix cores (v_mfma_f64_16x16x4), one 16 x 16 (a, b) tile per
//    wave, followed in registers by the b-sums with C over the tile.
// 3. k_vel_finish: sums the tile partials, forms v, updates x, raises flags,
//    and writes the per-CWF constant potential phases the propagation uses.
#include "icwf_plan.hpp"
#include "icwf_expi.hpp"

namespace icwf {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mfma_f64(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ void k_sinc(const double *__restrict__ pos, int Np, int n, double x_min, double h,
                       double *__restrict__ S, double *__restrict__ Sp, const int32_t *__restrict__ flags) {
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

// One wave per 16 (a) x 16 (b) tile; block = 4 waves = 32 x 32.  Lane l holds
// A = table[a0 + l%16][k], B = psi[b0 + l%16][k] with the k range split in
// four contiguous quarters by l/16.  Accumulator layout: lane l, register v
// holds D[mfma_row_f64(l, v)][l%16].
__global__ void __launch_bounds__(256) k_vel_gemm(const double *__restrict__ Sr, const double *__restrict__ Dr,
                                                  const double2 *__restrict__ psi1, int nr,
                                                  const double *__restrict__ SR, const double *__restrict__ DR,
                                                  const double2 *__restrict__ psi2, int nR,
                                                  const double2 *__restrict__ C, int Np,
                                                  double2 *__restrict__ part, const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int a0 = blockIdx.x * 32 + 16 * (wave >> 1);
    const int b0 = blockIdx.y * 32 + 16 * (wave & 1);
    const int row = lane & 15;
    const int quarter = lane >> 4;

    dbl4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0}, dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
    {
        const int q = nr >> 2;
        const double *ta = Sr + (size_t)(a0 + row) * nr + quarter * q;
        const double *td = Dr + (size_t)(a0 + row) * nr + quarter * q;
        const double2 *pb = psi1 + (size_t)(b0 + row) * nr + quarter * q;
        for (int s = 0; s < q; s += 2) {
            const double2 t = *reinterpret_cast<const double2 *>(ta + s);
            const double2 dd = *reinterpret_cast<const double2 *>(td + s);
            const double2 p0 = pb[s], p1 = pb[s + 1];
            ar = mfma_f64(t.x, p0.x, ar);
            ai = mfma_f64(t.x, p0.y, ai);
            dr = mfma_f64(dd.x, p0.x, dr);
            di = mfma_f64(dd.x, p0.y, di);
            ar = mfma_f64(t.y, p1.x, ar);
            ai = mfma_f64(t.y, p1.y, ai);
            dr = mfma_f64(dd.y, p1.x, dr);
            di = mfma_f64(dd.y, p1.y, di);
        }
    }
    dbl4 br = {0, 0, 0, 0}, bi = {0, 0, 0, 0}, er = {0, 0, 0, 0}, ei = {0, 0, 0, 0};
    {
        const int q = nR >> 2;
        const double *ta = SR + (size_t)(a0 + row) * nR + quarter * q;
        const double *td = DR + (size_t)(a0 + row) * nR + quarter * q;
        const double2 *pb = psi2 + (size_t)(b0 + row) * nR + quarter * q;
        for (int s = 0; s < q; s += 2) {
            const double2 t = *reinterpret_cast<const double2 *>(ta + s);
            const double2 dd = *reinterpret_cast<const double2 *>(td + s);
            const double2 p0 = pb[s], p1 = pb[s + 1];
            br = mfma_f64(t.x, p0.x, br);
            bi = mfma_f64(t.x, p0.y, bi);
            er = mfma_f64(dd.x, p0.x, er);
            ei = mfma_f64(dd.x, p0.y, ei);
            br = mfma_f64(t.y, p1.x, br);
            bi = mfma_f64(t.y, p1.y, bi);
            er = mfma_f64(dd.y, p1.x, er);
            ei = mfma_f64(dd.y, p1.y, ei);
        }
    }
    // epilogue: this lane holds column b = b0 + row, rows a = a0 + mfma_row_f64(lane, v)
    const double2 cb = C[b0 + row];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double2 A1 = make_double2(ar[v], ai[v]);
        const double2 D1 = make_double2(dr[v], di[v]);
        const double2 A2 = make_double2(br[v], bi[v]);
        const double2 D2 = make_double2(er[v], ei[v]);
        const double2 cA2 = cmul(cb, A2);
        double2 pPsi = cmul(cA2, A1);
        double2 pr = cmul(cA2, D1);
        double2 pR = cmul(cmul(cb, A1), D2);
        // sum over the 16 columns b held by lanes 16 quarter .. 16 quarter + 15
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
            const int a = a0 + mfma_row_f64(lane, v);
            double2 *dst = part + ((size_t)(b0 >> 4) * Np + a) * 3;
            dst[0] = pPsi;
            dst[1] = pr;
            dst[2] = pR;
        }
    }
}

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

__global__ void k_vel_finish(const double2 *__restrict__ part, int N, int Np, double m_r, double m_R, double dt,
                             const double *__restrict__ r, const double *__restrict__ R, double *__restrict__ r_new,
                             double *__restrict__ R_new, double *__restrict__ v_r, double *__restrict__ v_R,
                             double2 *__restrict__ psi_at, double r_lo, double r_hi, double R_lo, double R_hi,
                             ModelParams mp, double2 *__restrict__ cphase, int update, int32_t *__restrict__ flags,
                             unsigned long long *__restrict__ min_bits) {
    if (flags[kFlagHalt]) return;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    // the phases e^{-i V dt/2} of the one-coordinate potential part that is
    // constant on the grid of each CWF conditioned on this trajectory (V_2 at
    // R^a for the electronic CWF, V_1 at r^a for the nuclear one), at the
    // positions the propagation of this step conditions on
    cphase[a] = expi(-0.5 * dt * model_v2(mp, R[a]));
    cphase[Np + a] = expi(-0.5 * dt * model_v1(mp, r[a]));
    const int ntile = Np >> 4;
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
    v_r[a] = vr;
    v_R[a] = vR;
    if (update) {
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

__global__ void k_vel_reset(int32_t *flags, unsigned long long *min_bits) {
    if (threadIdx.x == 0) {
        flags[kFlagOut] = 0;
        *min_bits = 0x7ff0000000000000ULL;   // +inf
    }
}

}  // namespace

void launch_velocity(const Dims &d, const Bufs &b, bool update, hipStream_t s) {
    const int Np = padded(d.N);
    hipLaunchKernelGGL(k_sinc, dim3(Np), dim3(256), 0, s, b.r, Np, d.nr, d.r_min, d.hr, b.sinc_r, b.dsinc_r, b.flags);
    hipLaunchKernelGGL(k_sinc, dim3(Np), dim3(256), 0, s, b.R, Np, d.nR, d.R_min, d.hR, b.sinc_R, b.dsinc_R,
                       b.flags);
    hipLaunchKernelGGL(k_vel_gemm, dim3(Np / 32, Np / 32), dim3(256), 0, s, b.sinc_r, b.dsinc_r, b.psi1, d.nr,
                       b.sinc_R, b.dsinc_R, b.psi2, d.nR, b.C, Np, b.vpart, b.flags);
    unsigned long long *min_bits = reinterpret_cast<unsigned long long *>(b.scal);
    hipLaunchKernelGGL(k_vel_reset, dim3(1), dim3(64), 0, s, b.flags, min_bits);
    const double r_hi = d.r_min + d.hr * d.nr, R_hi = d.R_min + d.hR * d.nR;
    hipLaunchKernelGGL(k_vel_finish, dim3((d.N + 255) / 256), dim3(256), 0, s, b.vpart, d.N, Np, d.m_r, d.m_R,
                       d.dt, b.r, b.R, b.r_new, b.R_new, b.v_r, b.v_R, b.psi_at, d.r_min, r_hi, d.R_min, R_hi, d.mp,
                       b.cphase, update ? 1 : 0, b.flags, min_bits);
}

}  // namespace icwf
