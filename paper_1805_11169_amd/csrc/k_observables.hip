// Observables of the ansatz (text around the Shin-Metiu figure): the norm
// C^H S C, the reduced densities
//     rho(R_j) = sum_{b,a} conj(C_b psi2^b_j) S1[b][a] C_a psi2^a_j
//     rho(r_i) = sum_{b,a} conj(C_b psi1^b_i) S2[b][a] C_a psi1^a_i,
// the BO projections chi^(n)(R_j) = sum_a C_a psi2^a_j <phi_n(.;R_j)|psi1^a>,
// the populations P_n = hR sum_j |chi^(n)_j|^2 and the decoherence indicator
// D_nm = hR sum_j |chi^(n)_j|^2 |chi^(m)_j|^2.  Computed on demand, not every step.
// Output layout: [norm, rho_r[nr], rho_R[nR], pop[n_bo], D[n_bo][n_bo]].
#include "icwf_plan.hpp"

namespace icwf {

namespace {

__device__ inline double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// out[0] = Re(C^H S C); one block of 256 threads, one thread per row strip.
__global__ void k_obs_norm(const double2 *__restrict__ S, const double2 *__restrict__ C, int Np,
                           double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < Np; b += blockDim.x) {
        double2 y = make_double2(0, 0);
        const double2 *row = S + (size_t)b * Np;
        for (int a = 0; a < Np; ++a) y = cadd(y, cmul(row[a], C[a]));
        acc += cmulc(C[b], y).x;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[0] = s;
}

// U[a][i] = C_a psi[a][i]
__global__ void k_obs_u(const double2 *__restrict__ psi, const double2 *__restrict__ C, int n, int Np,
                        double2 *__restrict__ U) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Np * n) return;
    U[idx] = cmul(C[idx / n], psi[idx]);
}

// rho[j] = Re sum_b conj(U[b][j]) sum_a O[b][a] U[a][j]; one block per j.
__global__ void k_obs_density(const double2 *__restrict__ O, const double2 *__restrict__ U, int n, int Np,
                              double *__restrict__ rho) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < Np; b += blockDim.x) {
        const double2 *row = O + (size_t)b * Np;
        double2 v = make_double2(0, 0);
        for (int a = 0; a < Np; ++a) v = cadd(v, cmul(row[a], U[(size_t)a * n + j]));
        acc += cmulc(U[(size_t)b * n + j], v).x;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) rho[j] = s;
}

// chi[nb][j] = sum_a C_a psi2[a][j] hr sum_i bo[j][nb][i] psi1[a][i]; one block per (j, nb).
__global__ void k_obs_chi(const double *__restrict__ bo, const double2 *__restrict__ psi1,
                          const double2 *__restrict__ psi2, const double2 *__restrict__ C, int nr, int nR,
                          int n_bo, int Np, double hr, double2 *__restrict__ chi) {
    __shared__ double red[256];
    const int j = blockIdx.x, nb = blockIdx.y;
    const double *phi = bo + ((size_t)j * n_bo + nb) * nr;
    double2 acc = make_double2(0, 0);
    for (int a = threadIdx.x; a < Np; a += blockDim.x) {
        const double2 *p = psi1 + (size_t)a * nr;
        double2 pr = make_double2(0, 0);
        for (int i = 0; i < nr; ++i) pr = cadd(pr, cscale(p[i], phi[i]));
        acc = cadd(acc, cmul(cmul(C[a], psi2[(size_t)a * nR + j]), cscale(pr, hr)));
    }
    const double sr = block_sum(acc.x, red);
    const double si = block_sum(acc.y, red);
    if (threadIdx.x == 0) chi[(size_t)nb * nR + j] = make_double2(sr, si);
}

// pop[n] and D[n][m]; one block.
__global__ void k_obs_pop(const double2 *__restrict__ chi, int nR, int n_bo, double hR, double *__restrict__ pop,
                          double *__restrict__ D) {
    __shared__ double red[256];
    for (int n = 0; n < n_bo; ++n) {
        for (int m = 0; m <= n; ++m) {
            double acc = 0.0;
            for (int j = threadIdx.x; j < nR; j += blockDim.x) {
                const double2 cn = chi[(size_t)n * nR + j], cm = chi[(size_t)m * nR + j];
                const double dn = cn.x * cn.x + cn.y * cn.y, dm = cm.x * cm.x + cm.y * cm.y;
                acc += (n == m) ? dn : dn * dm;
            }
            // P_n from the m == n pass, D_nn from a separate sum of dn^2
            const double s = block_sum(acc, red);
            if (n == m) {
                double acc2 = 0.0;
                for (int j = threadIdx.x; j < nR; j += blockDim.x) {
                    const double2 cn = chi[(size_t)n * nR + j];
                    const double dn = cn.x * cn.x + cn.y * cn.y;
                    acc2 += dn * dn;
                }
                const double s2 = block_sum(acc2, red);
                if (threadIdx.x == 0) {
                    pop[n] = hR * s;
                    D[n * n_bo + n] = hR * s2;
                }
            } else if (threadIdx.x == 0) {
                D[n * n_bo + m] = hR * s;
                D[m * n_bo + n] = hR * s;
            }
        }
    }
}

}  // namespace

void launch_observables(const Dims &d, const Bufs &b, int parity, hipStream_t s) {
    const int Np = padded(d.N);
    double *out = b.obs_out;
    hipLaunchKernelGGL(k_obs_norm, dim3(1), dim3(256), 0, s, b.Smat[parity], b.C, Np, out);
    size_t tot = (size_t)Np * d.nR;
    hipLaunchKernelGGL(k_obs_u, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b.psi2, b.C, d.nR, Np,
                       b.obs_u);
    hipLaunchKernelGGL(k_obs_density, dim3(d.nR), dim3(256), 0, s, b.S1, b.obs_u, d.nR, Np, out + 1 + d.nr);
    tot = (size_t)Np * d.nr;
    hipLaunchKernelGGL(k_obs_u, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b.psi1, b.C, d.nr, Np,
                       b.obs_u);
    hipLaunchKernelGGL(k_obs_density, dim3(d.nr), dim3(256), 0, s, b.S2, b.obs_u, d.nr, Np, out + 1);
    if (d.n_bo > 0) {
        hipLaunchKernelGGL(k_obs_chi, dim3(d.nR, d.n_bo), dim3(256), 0, s, b.bo, b.psi1, b.psi2, b.C, d.nr, d.nR,
                           d.n_bo, Np, d.hr, b.obs_chi);
        double *pop = out + 1 + d.nr + d.nR;
        hipLaunchKernelGGL(k_obs_pop, dim3(1), dim3(256), 0, s, b.obs_chi, d.nR, d.n_bo, d.hR, pop, pop + d.n_bo);
    }
}

}  // namespace icwf
