// Observables of the ansatz (text around the Shin-Metiu figure), all from the
// wavefunction on the grid, Eq. 7 evaluated at the grid points:
//     Psi(r_i, R_j) = sum_a C_a psi1^a_i psi2^a_j          (one complex GEMM)
//     rho(r_i) = hR sum_j |Psi_ij|^2,   rho(R_j) = hr sum_i |Psi_ij|^2,
//     norm = hr sum_i rho(r_i)  (= C^H S C),
//     chi^(n)(R_j) = hr sum_i phi_n(r_i; R_j) Psi_ij  (BO projections, real phi_n),
//     P_n = hR sum_j |chi^(n)_j|^2,  D_nm = hR sum_j |chi^(n)_j|^2 |chi^(m)_j|^2.
// The GEMM costs N n_r n_R complex products, against N^2 (n_r + n_R) for the
// same densities written with the single-species overlaps.  Computed on
// demand, not every step; every sum runs in a fixed order (bitwise
// repeatable).  Output layout: [norm, rho_r[nr], rho_R[nR], pop[n_bo], D[n_bo][n_bo]].
#include "icwf_plan.hpp"

namespace icwf {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Psi = U^T V, U[a][i] = C_a psi1[a][i], V[a][j] = psi2[a][j], a < Np.  One
// 64 x 64 tile of Psi per work-group of 4 waves, wave w on the 32 x 32
// quarter (rows 32 (w / 2), columns 32 (w % 2)) as 2 x 2 fragments of
// v_mfma_f64_16x16x4 with rows = i, columns = j and the trajectory a as the
// reduction index.  16-trajectory chunks of U (times C_a) and V are staged
// through double-buffered LDS by coalesced row loads (64 consecutive grid
// points per row).  Rows or columns beyond the grid (n = 32) read zeros and
// are not stored.
constexpr int kOT = 64, kOKC = 16, kOLD = kOT + 1;

__global__ void __launch_bounds__(256) k_obs_psi(const double2 *__restrict__ psi1, const double2 *__restrict__ psi2,
                                                 const double2 *__restrict__ C, int nr, int nR, int Np,
                                                 double2 *__restrict__ Psi) {
    __shared__ double2 sU[2][kOKC][kOLD];
    __shared__ double2 sV[2][kOKC][kOLD];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int row = lane & 15, quarter = lane >> 4;
    const int i0 = blockIdx.y * kOT, j0 = blockIdx.x * kOT;
    const int wi = 32 * (wave >> 1), wj = 32 * (wave & 1);
    // staging: thread t loads grid point c = t % 64 of the chunk rows t / 64 + 4 m
    const int sc = t & 63, sr = t >> 6;
    const bool ui = i0 + sc < nr, vj = j0 + sc < nR;
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            re[f][g] = dbl4{0, 0, 0, 0};
            im[f][g] = dbl4{0, 0, 0, 0};
        }
    double2 ru[4], rv[4];
    auto load = [&](int a0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int a = a0 + sr + 4 * m;
            ru[m] = ui ? cmul(C[a], psi1[(size_t)a * nr + i0 + sc]) : make_double2(0.0, 0.0);
            rv[m] = vj ? psi2[(size_t)a * nR + j0 + sc] : make_double2(0.0, 0.0);
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            sU[buf][sr + 4 * m][sc] = ru[m];
            sV[buf][sr + 4 * m][sc] = rv[m];
        }
    };
    load(0);
    stage(0);
    __syncthreads();
    const int nch = Np / kOKC;
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) load((ch + 1) * kOKC);
#pragma unroll
        for (int s4 = 0; s4 < kOKC / 4; ++s4) {
            const int kk = 4 * s4 + quarter;
            double2 uv[2], vv[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                uv[f] = sU[buf][kk][wi + 16 * f + row];
                vv[f] = sV[buf][kk][wj + 16 * f + row];
            }
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    // u v = (ur vr - ui vi) + i (ur vi + ui vr)
                    re[f][g] = mfma(uv[f].x, vv[g].x, re[f][g]);
                    re[f][g] = mfma(-uv[f].y, vv[g].y, re[f][g]);
                    im[f][g] = mfma(uv[f].x, vv[g].y, im[f][g]);
                    im[f][g] = mfma(uv[f].y, vv[g].x, im[f][g]);
                }
        }
        if (more) stage(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + 16 * f + mfma_row_f64(lane, v);
                const int j = j0 + wj + 16 * g + row;
                if (i < nr && j < nR) Psi[(size_t)i * nR + j] = make_double2(re[f][g][v], im[f][g][v]);
            }
}

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

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// rho_r[i] = hR sum_j |Psi_ij|^2: one wave per row, four rows per block.
__global__ void k_obs_rho_r(const double2 *__restrict__ Psi, int nr, int nR, double hR, double *__restrict__ rho) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= nr) return;
    double acc = 0.0;
    for (int j = lane; j < nR; j += 64) {
        const double2 p = Psi[(size_t)i * nR + j];
        acc += p.x * p.x + p.y * p.y;
    }
    acc = wave_sum(acc);
    if (lane == 0) rho[i] = hR * acc;
}

// rho_R[j] = hr sum_i |Psi_ij|^2 in two passes, so that tall grids fill the
// device: block (x, y) sums rows y nr/S ... (y + 1) nr/S - 1 of 64 columns
// (four row slices reduced in LDS in a fixed order) into part[y][j]; then
// the S partial sums of each column are added in order.
__global__ void k_obs_rho_R_part(const double2 *__restrict__ Psi, int nr, int nR, double *__restrict__ part) {
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + c;
    const int rows = nr / kRhoSlices, i0 = blockIdx.y * rows;
    double acc = 0.0;
    if (j < nR)
        for (int i = i0 + sl; i < i0 + rows; i += 4) {
            const double2 p = Psi[(size_t)i * nR + j];
            acc += p.x * p.x + p.y * p.y;
        }
    red[sl][c] = acc;
    __syncthreads();
    if (sl == 0 && j < nR) part[(size_t)blockIdx.y * nR + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void k_obs_rho_R_sum(const double *__restrict__ part, int nR, double hr, double *__restrict__ rho) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nR) return;
    double acc = 0.0;
    for (int s = 0; s < kRhoSlices; ++s) acc += part[(size_t)s * nR + j];
    rho[j] = hr * acc;
}

// out[0] = hr sum_i rho_r[i]; one block.
__global__ void k_obs_norm(const double *__restrict__ rho_r, int nr, double hr, double *__restrict__ out) {
    __shared__ double part[4];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nr; i += blockDim.x) acc += rho_r[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = hr * (((part[0] + part[1]) + part[2]) + part[3]);
}

// chi[nb][j] = hr sum_i bo[j][nb][i] Psi_ij: one wave per (j, nb).
__global__ void k_obs_chi(const double *__restrict__ bo, const double2 *__restrict__ Psi, int nr, int nR,
                          int n_bo, double hr, double2 *__restrict__ chi) {
    const int j = blockIdx.x, nb = blockIdx.y, lane = threadIdx.x;
    const double *phi = bo + ((size_t)j * n_bo + nb) * nr;
    double sr = 0.0, si = 0.0;
    for (int i = lane; i < nr; i += 64) {
        const double2 p = Psi[(size_t)i * nR + j];
        sr += phi[i] * p.x;
        si += phi[i] * p.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) chi[(size_t)nb * nR + j] = make_double2(hr * sr, hr * si);
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

void launch_grid_observables(const double2 *Psi, int nr, int nR, double hr, double hR, int n_bo, const double *bo,
                             double2 *chi, double *part, double *out, hipStream_t s) {
    double *rho_r = out + 1, *rho_R = out + 1 + nr;
    hipLaunchKernelGGL(k_obs_rho_r, dim3((nr + 3) / 4), dim3(256), 0, s, Psi, nr, nR, hR, rho_r);
    hipLaunchKernelGGL(k_obs_rho_R_part, dim3((nR + 63) / 64, kRhoSlices), dim3(256), 0, s, Psi, nr, nR, part);
    hipLaunchKernelGGL(k_obs_rho_R_sum, dim3((nR + 255) / 256), dim3(256), 0, s, part, nR, hr, rho_R);
    hipLaunchKernelGGL(k_obs_norm, dim3(1), dim3(256), 0, s, rho_r, nr, hr, out);
    if (n_bo > 0) {
        hipLaunchKernelGGL(k_obs_chi, dim3(nR, n_bo), dim3(64), 0, s, bo, Psi, nr, nR, n_bo, hr, chi);
        double *pop = out + 1 + nr + nR;
        hipLaunchKernelGGL(k_obs_pop, dim3(1), dim3(256), 0, s, chi, nR, n_bo, hR, pop, pop + n_bo);
    }
}

void launch_observables(const Dims &d, const Bufs &b, hipStream_t s) {
    const int Np = padded(d.N);
    const dim3 tiles((d.nR + kOT - 1) / kOT, (d.nr + kOT - 1) / kOT);
    hipLaunchKernelGGL(k_obs_psi, tiles, dim3(256), 0, s, b.psi1, b.psi2, b.C, d.nr, d.nR, Np, b.obs_psi);
    launch_grid_observables(b.obs_psi, d.nr, d.nR, d.hr, d.hR, d.n_bo, b.bo, b.obs_chi, b.obs_part, b.obs_out, s);
}

}  // namespace icwf
