// Crank-Nicolson step of every CWF of one species (Eqs. 5-6 with the
// conditioning frozen at the start of the step), the propagator a user can
// select instead of the split operator:
//
//     (1 + i dt/2 H) psi_new = (1 - i dt/2 H) psi,   H = -(1/2m) D2 + W(., x^a),
//
// D2 the periodic three-point second difference.  The system is cyclic
// tridiagonal, a_i = c_i = -i dt / (4 m h^2), b_i = 1 + i dt/2 (1/(m h^2) + V_i).
// One work-group per CWF solves it by parallel cyclic reduction in LDS: at
// stride s every equation i eliminates x_{i-s} and x_{i+s} with equations
// i - s and i + s (indices mod n); after log2 n steps the stride is n, the
// equation reads (a_i + b_i + c_i) x_i = d_i.  With n a power of two the
// periodic wrap needs no special case (at stride n/2 both neighbours are the
// same equation, and the step is the elimination of a 2 x 2 system).  No
// pivoting is needed: A = 1 + i dt/2 H with H real symmetric has the identity
// as its Hermitian part, every system the reduction forms (for each residue
// class of the stride, a Schur complement of A) has a Hermitian part of at
// least the identity, so every pivot has a real part of at least 1.  The
// systems need not be diagonally dominant (on the cavity grid dt/(2 m h^2) =
// 5.2 exceeds |b_i| where the tilted potential falls below -1.9).
// Grids up to 2048 points (four n-point complex arrays: 128 KB of LDS).

#include <hip/hip_runtime.h>

#include "icwf_device.hpp"
#include "icwf_plan.hpp"

namespace icwf {
namespace {

template <int L>
constexpr int cn_threads() {
    return (1 << L) < 1024 ? (1 << L) : 1024;
}

__device__ inline double2 cdiv(double2 a, double2 b) {
    const double inv = 1.0 / (b.x * b.x + b.y * b.y);
    return make_double2((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);
}

// psi [Np][n] in place; cond [Np] the other species' coordinate of each CWF
// (species 1: R^a; species 2: r^a); psi_f32 (or null) gets an FP32 copy.
template <int LOG2N>
__global__ void __launch_bounds__(cn_threads<LOG2N>()) k_propagate_cn(double2 *__restrict__ psi,
                                                                      const double *__restrict__ cond, int species,
                                                                      double x_min, double h, double m, double dt,
                                                                      ModelParams mp, float2 *__restrict__ psi_f32,
                                                                      const int32_t *__restrict__ flags, const long long *__restrict__ zoff, const ModelParams *__restrict__ mpd) {
    const long long zo_ = batch_offset(zoff);
    psi = zshift(psi, zo_);
    cond = zshift(cond, zo_);
    psi_f32 = zshift(psi_f32, zo_);
    flags = zshift(flags, zo_);
    if (zoff) mp = *zshift(mpd, zo_);

    if (flags[kFlagHalt]) return;
    constexpr int n = 1 << LOG2N, nt = cn_threads<LOG2N>(), E = n / nt;
    __shared__ double2 sa[n], sb[n], sc[n], sd[n];
    const size_t row = (size_t)blockIdx.x * n;
    const double xc = cond[blockIdx.x];
    const double kin = 1.0 / (m * h * h), t = 0.5 * dt;
    const double2 off = make_double2(0.0, -0.5 * t * kin);     // -i dt / (4 m h^2)
    double V[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x + e * nt;
        const double x = x_min + i * h;
        V[e] = species == 1 ? model_w(mp, x, xc) : model_w(mp, xc, x);
        sd[i] = psi[row + i];
    }
    __syncthreads();
    // right-hand side (1 - i t H) psi and the matrix
    double2 rhs[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x + e * nt;
        const double2 p = sd[i], pl = sd[(i - 1) & (n - 1)], pr = sd[(i + 1) & (n - 1)];
        const double dg = kin + V[e];
        // H psi = dg psi - (psi_{i-1} + psi_{i+1}) kin / 2
        const double hx = dg * p.x - 0.5 * kin * (pl.x + pr.x), hy = dg * p.y - 0.5 * kin * (pl.y + pr.y);
        rhs[e] = make_double2(p.x + t * hy, p.y - t * hx);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x + e * nt;
        sa[i] = off;
        sc[i] = off;
        sb[i] = make_double2(1.0, t * (kin + V[e]));
        sd[i] = rhs[e];
    }
    __syncthreads();
    for (int s = 1; s < n; s <<= 1) {
        double2 na[E], nb[E], nc[E], nd[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = threadIdx.x + e * nt, im = (i - s) & (n - 1), ip = (i + s) & (n - 1);
            const double2 al = cdiv(make_double2(-sa[i].x, -sa[i].y), sb[im]);
            const double2 ga = cdiv(make_double2(-sc[i].x, -sc[i].y), sb[ip]);
            na[e] = cmul(al, sa[im]);
            nc[e] = cmul(ga, sc[ip]);
            nb[e] = cadd(sb[i], cadd(cmul(al, sc[im]), cmul(ga, sa[ip])));
            nd[e] = cadd(sd[i], cadd(cmul(al, sd[im]), cmul(ga, sd[ip])));
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = threadIdx.x + e * nt;
            sa[i] = na[e];
            sb[i] = nb[e];
            sc[i] = nc[e];
            sd[i] = nd[e];
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = threadIdx.x + e * nt;
        const double2 x = cdiv(sd[i], cadd(sa[i], cadd(sb[i], sc[i])));
        psi[row + i] = x;
        if (psi_f32) psi_f32[row + i] = make_float2((float)x.x, (float)x.y);
    }
}

template <int L>
void launch_cn(const Dims &d, const Bufs &b, int species, hipStream_t s) {
    const int Np = padded(d.N);
    if (species == 1)
        hipLaunchKernelGGL(k_propagate_cn<L>, dim3(Np, 1, d.batch), dim3(cn_threads<L>()), 0, s, b.psi1, b.R, 1,
                           d.r_min, d.hr, d.m_r, d.dt, d.mp, d.prec == 1 && d.fp32_residual ? b.psi1_f32 : nullptr,
                           b.flags, d.zoff, d.mpd);
    else
        hipLaunchKernelGGL(k_propagate_cn<L>, dim3(Np, 1, d.batch), dim3(cn_threads<L>()), 0, s, b.psi2, b.r, 2,
                           d.R_min, d.hR, d.m_R, d.dt, d.mp, nullptr, b.flags, d.zoff, d.mpd);
}

}  // namespace

void launch_propagate_cn(const Dims &d, const Bufs &b, int species, hipStream_t s) {
    const int n = species == 1 ? d.nr : d.nR;   // validated at creation: a power of two in [32, 2048]
    switch (n) {
    case 32: launch_cn<5>(d, b, species, s); break;
    case 64: launch_cn<6>(d, b, species, s); break;
    case 128: launch_cn<7>(d, b, species, s); break;
    case 256: launch_cn<8>(d, b, species, s); break;
    case 512: launch_cn<9>(d, b, species, s); break;
    case 1024: launch_cn<10>(d, b, species, s); break;
    case 2048: launch_cn<11>(d, b, species, s); break;
    default: break;
    }
}

}  // namespace icwf
