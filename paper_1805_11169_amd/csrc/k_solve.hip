// Assembly of S and K = W - W1 - W2 (Eqs. 8-9), the Tikhonov-regularised
// Cholesky factorisation of S + eps I, and RK4 for i S dC/dt = K C.
//
// Assembly.  With W = V_1(r) + V_2(R) + W_c(r, R), the one-coordinate parts of
// Eq. 9b cancel against Eqs. 9c-9d except at the ket's own trajectory:
//     K[b][a] = Wc[b][a] - E1[b][a] S2[b][a] - S1[b][a] E2[b][a]
//               - (V_1(r^a) + V_2(R^a)) S[b][a],     S = S1 o S2,
// where Wc, E1, E2 are the Eq. 9b-9d integrals with W_c alone.  Per step the
// kernel forms S_k+1, K^- = K(psi_k+1, x_k) (end of the step just taken),
// K_k+1 = K(psi_k+1, x_k+1) (start of the next), the midpoint averages, and
// the regularised matrices handed to the factorisation.
//
// Cholesky (lower, in place, two matrices per launch): right-looking with
// 64-wide panels.  k_chol_panel factors the 64 x 64 diagonal block in LDS (every
// work-group redundantly; work-group 0 stores it) and solves its 64 rows of
// the panel, x L11^H = a, one row per lane.  k_chol_update subtracts
// L21 L21^H from the trailing lower triangle on FP64 matrix cores.  A pivot
// that is not positive raises the solve flag and halts the step.
//
// RK4 (classical, S and K linear in time between the step ends, so the
// midpoint is their average): each stage is a matvec K v over many
// work-groups, then one work-group solves L L^H z = K v by blocked forward and
// back substitution in LDS and applies the stage update k = -i z.
#include "icwf_plan.hpp"

namespace icwf {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ assembly
__global__ void k_assemble(const double2 *__restrict__ S1, const double2 *__restrict__ S2,
                           const double2 *__restrict__ E1a, const double2 *__restrict__ E1b,
                           const double2 *__restrict__ E2a, const double2 *__restrict__ E2b,
                           const double2 *__restrict__ Wc, const double2 *__restrict__ Scur,
                           const double2 *__restrict__ Kcur, const double *__restrict__ r,
                           const double *__restrict__ R, const double *__restrict__ r_new,
                           const double *__restrict__ R_new, ModelParams mp, int N, int Np, double eps,
                           int initial, double2 *__restrict__ Snext, double2 *__restrict__ Kminus,
                           double2 *__restrict__ Knext, double2 *__restrict__ Amid, double2 *__restrict__ Anext,
                           double2 *__restrict__ Kmid, const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Np * Np) return;
    const int b = (int)(idx / Np), a = (int)(idx - (size_t)b * Np);
    const double2 s1 = S1[idx], s2 = S2[idx];
    const double2 S = cmul(s1, s2);
    const double2 w = (b <= a) ? Wc[idx] : cconj(Wc[(size_t)a * Np + b]);
    double ca = 0.0, cn = 0.0;
    if (a < N) {
        ca = model_v1(mp, r[a]) + model_v2(mp, R[a]);
        cn = model_v1(mp, r_new[a]) + model_v2(mp, R_new[a]);
    }
    const double reg = (a == b) ? eps : 0.0;
    if (initial) {
        // start of the run: S_0, K_0 = K(psi_0, x_0) -> next slots of parity 0 == current
        Snext[idx] = S;
        Knext[idx] = csub(csub(csub(w, cmul(E1a[idx], s2)), cmul(s1, E2a[idx])), cscale(S, ca));
        Anext[idx] = make_double2(S.x + reg, S.y);
        return;
    }
    const double2 km = csub(csub(csub(w, cmul(E1a[idx], s2)), cmul(s1, E2a[idx])), cscale(S, ca));
    const double2 kn = csub(csub(csub(w, cmul(E1b[idx], s2)), cmul(s1, E2b[idx])), cscale(S, cn));
    const double2 sc = Scur[idx];
    Snext[idx] = S;
    Kminus[idx] = km;
    Knext[idx] = kn;
    Anext[idx] = make_double2(S.x + reg, S.y);
    Amid[idx] = make_double2(0.5 * (sc.x + S.x) + reg, 0.5 * (sc.y + S.y));
    const double2 kc = Kcur[idx];
    Kmid[idx] = make_double2(0.5 * (kc.x + km.x), 0.5 * (kc.y + km.y));
}

// ------------------------------------------------------------------ Cholesky
constexpr int NB = kCholNb;   // 64

__device__ inline void raise_solve(int32_t *flags) {
    atomicOr(&flags[kFlagSolve], 1);
    atomicOr(&flags[kFlagHalt], 1);
}

// Factor the NB x NB diagonal block (lower) held in LDS tile[NB][NB]; 64 threads.
__device__ void factor_diag(double2 (*tile)[NB], int32_t *flags) {
    const int t = threadIdx.x;
    for (int j = 0; j < NB; ++j) {
        double d = tile[j][j].x;
        if (!(d > 0.0)) {                       // not positive definite (or NaN)
            if (t == 0) raise_solve(flags);
            d = 1.0;
        }
        d = sqrt(d);
        __syncthreads();
        if (t == j) tile[j][j] = make_double2(d, 0.0);
        if (t > j) tile[t][j] = cscale(tile[t][j], 1.0 / d);
        __syncthreads();
        // trailing update of column k = t (rows i >= k): tile[i][k] -= L[i][j] conj(L[k][j])
        if (t > j) {
            const double2 lkj = cconj(tile[t][j]);
            for (int i = t; i < NB; ++i) tile[i][t] = csub(tile[i][t], cmul(tile[i][j], lkj));
        }
        __syncthreads();
    }
}

// The factored diagonal block goes to a scratch tile, not into A: other
// work-groups of the same launch may still be reading the unfactored block.
// Work-group 0 of the next launch (or k_chol_flush after the last panel) copies
// it into place.
__global__ void __launch_bounds__(64) k_chol_panel(double2 *A0, double2 *A1, int Np, int kb,
                                                   double2 *__restrict__ diag, int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    __shared__ double2 tile[NB][NB];
    double2 *A = blockIdx.y ? A1 : A0;
    double2 *D = diag + (size_t)blockIdx.y * NB * NB;
    const int t = threadIdx.x;
    if (blockIdx.x == 0 && kb > 0) {
        const int pb = kb - NB;
        for (int i = 0; i < NB; ++i)
            if (t <= i) A[(size_t)(pb + i) * Np + pb + t] = D[i * NB + t];
    }
    for (int i = 0; i < NB; ++i) tile[i][t] = A[(size_t)(kb + i) * Np + kb + t];
    __syncthreads();
    factor_diag(tile, flags);
    if (blockIdx.x == 0) {
        for (int i = 0; i < NB; ++i) D[i * NB + t] = tile[i][t];
    }
    // rows of the panel below the block: x L11^H = a, column by column
    // (right-looking): x_j = a_j / L11[j][j], then a_k -= x_j conj(L11[k][j])
    // for k > j.  Only the not yet solved part of the row stays live.
    const int i = kb + NB + blockIdx.x * 64 + t;
    if (i >= Np) return;
    double2 *arow = A + (size_t)i * Np + kb;
    double2 a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] = arow[j];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const double2 xj = cscale(a[j], 1.0 / tile[j][j].x);
        arow[j] = xj;
#pragma unroll
        for (int k = j + 1; k < NB; ++k) a[k] = csub(a[k], cmul(xj, cconj(tile[k][j])));
    }
}

__global__ void __launch_bounds__(64) k_chol_flush(double2 *A0, double2 *A1, int Np, int kb,
                                                   const double2 *__restrict__ diag,
                                                   const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    double2 *A = blockIdx.y ? A1 : A0;
    const double2 *D = diag + (size_t)blockIdx.y * NB * NB;
    const int t = threadIdx.x;
    for (int i = 0; i < NB; ++i)
        if (t <= i) A[(size_t)(kb + i) * Np + kb + t] = D[i * NB + t];
}

// Trailing update A[i][k] -= sum_j L[i][j] conj(L[k][j]) over the lower
// triangle i >= k of rows/cols kb+NB .. Np-1, j over the panel; one wave per
// 32 x 32 tile.
__global__ void __launch_bounds__(64) k_chol_update(double2 *A0, double2 *A1, int Np, int kb,
                                                    const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    double2 *A = blockIdx.y ? A1 : A0;
    const int t = blockIdx.x;
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tk = t - ti * (ti + 1) / 2;
    const int base = kb + NB;
    const int i0 = base + 32 * ti, k0 = base + 32 * tk;
    const int lane = threadIdx.x, row = lane & 15, quarter = lane >> 4;
    const int q = NB / 4;
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            re[f][g] = dbl4{0, 0, 0, 0};
            im[f][g] = dbl4{0, 0, 0, 0};
        }
    const double2 *xp[2], *yp[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        xp[f] = A + (size_t)(i0 + 16 * f + row) * Np + kb + quarter * q;
        yp[f] = A + (size_t)(k0 + 16 * f + row) * Np + kb + quarter * q;
    }
    for (int s = 0; s < q; ++s) {
        double2 xv[2], yv[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            xv[f] = xp[f][s];
            yv[f] = yp[f][s];
        }
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                // x conj(y) = (xr yr + xi yi) + i (xi yr - xr yi)
                re[f][g] = mfma(xv[f].x, yv[g].x, re[f][g]);
                re[f][g] = mfma(xv[f].y, yv[g].y, re[f][g]);
                im[f][g] = mfma(xv[f].y, yv[g].x, im[f][g]);
                im[f][g] = mfma(-xv[f].x, yv[g].y, im[f][g]);
            }
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = i0 + 16 * f + mfma_row_f64(lane, v);
                const int kk = k0 + 16 * g + row;
                double2 *p = A + (size_t)ii * Np + kk;
                const double2 o = *p;
                *p = make_double2(o.x - re[f][g][v], o.y - im[f][g][v]);
            }
}

// ------------------------------------------------------------------ RK4
// y = M v, one wave per row.
__global__ void __launch_bounds__(256) k_matvec(const double2 *__restrict__ M, const double2 *__restrict__ v,
                                                double2 *__restrict__ y, int Np,
                                                const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    const int lane = threadIdx.x & 63;
    const int rowi = blockIdx.x * 4 + (threadIdx.x >> 6);
    const double2 *m = M + (size_t)rowi * Np;
    double2 acc = make_double2(0, 0);
    for (int c = lane; c < Np; c += 64) acc = cadd(acc, cmul(m[c], v[c]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off);
        acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) y[rowi] = acc;
}

// Solve L L^H z = z in place (z in LDS), L lower Np x Np; 1024 threads.
__device__ void chol_solve(const double2 *__restrict__ L, int Np, double2 *z, double2 (*red)[64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;   // 16 waves
    // forward: L w = z
    for (int B = 0; B < Np; B += 64) {
        // partial sums over the columns left of the block: 4 rows per wave
        for (int rr = 0; rr < 4; ++rr) {
            const int i = B + 4 * wave + rr;
            const double2 *Li = L + (size_t)i * Np;
            double2 acc = make_double2(0, 0);
            for (int c = lane; c < B; c += 64) acc = cadd(acc, cmul(Li[c], z[c]));
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                acc.x += __shfl_xor(acc.x, off);
                acc.y += __shfl_xor(acc.y, off);
            }
            if (lane == 0) red[0][4 * wave + rr] = acc;
        }
        __syncthreads();
        if (wave == 0) {
            double2 tv = csub(z[B + lane], red[0][lane]);
            const double2 *Lrow = L + (size_t)(B + lane) * Np + B;
            for (int jj = 0; jj < 64; ++jj) {
                double2 xj = make_double2(0, 0);
                if (lane == jj) xj = cscale(tv, 1.0 / Lrow[jj].x);
                xj.x = __shfl(xj.x, jj);
                xj.y = __shfl(xj.y, jj);
                if (lane > jj) tv = csub(tv, cmul(Lrow[jj], xj));
                if (lane == jj) tv = xj;
            }
            z[B + lane] = tv;
        }
        __syncthreads();
    }
    // backward: L^H x = w
    for (int B = Np - 64; B >= 0; B -= 64) {
        double2 acc = make_double2(0, 0);
        for (int i = B + 64 + wave; i < Np; i += 16) acc = cadd(acc, cmul(cconj(L[(size_t)i * Np + B + lane]), z[i]));
        red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0) {
            double2 u = z[B + lane];
            for (int w = 0; w < 16; ++w) u = csub(u, red[w][lane]);
            for (int jj = 63; jj >= 0; --jj) {
                const double2 *Lrow = L + (size_t)(B + jj) * Np + B;
                double2 xj = make_double2(0, 0);
                if (lane == jj) xj = cscale(u, 1.0 / Lrow[jj].x);
                xj.x = __shfl(xj.x, jj);
                xj.y = __shfl(xj.y, jj);
                if (lane < jj) u = csub(u, cmul(cconj(Lrow[lane]), xj));
                if (lane == jj) u = xj;
            }
            z[B + lane] = u;
        }
        __syncthreads();
    }
}

constexpr int kSolveLdsMax = 3072;

// stage: 1..4 of RK4; 0 = initial coefficients (C = solve(y)).
__global__ void __launch_bounds__(1024) k_rk_stage(const double2 *__restrict__ L, double2 *__restrict__ y,
                                                   int stage, double dt, int N, int Np, double2 *__restrict__ C,
                                                   double2 *__restrict__ Cacc, double2 *__restrict__ Cstage,
                                                   double *__restrict__ r, double *__restrict__ R,
                                                   const double *__restrict__ r_new,
                                                   const double *__restrict__ R_new, int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    extern __shared__ double2 zlds[];
    __shared__ double2 red[16][64];
    // z lives in LDS when it fits beside red (64 KB per work-group), else in
    // the y buffer itself (global memory; the block barrier orders it).
    double2 *zs = (Np <= kSolveLdsMax) ? zlds : const_cast<double2 *>(y);
    if (Np <= kSolveLdsMax) {
        for (int i = threadIdx.x; i < Np; i += blockDim.x) zs[i] = y[i];
    }
    __syncthreads();
    chol_solve(L, Np, zs, red);
    int bad = 0;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) {
        const double2 z = zs[i];
        if (stage == 0) {
            C[i] = (i < N) ? z : make_double2(0, 0);
            bad |= !(isfinite(z.x) && isfinite(z.y));
            continue;
        }
        const double2 k = make_double2(z.y, -z.x);   // -i z
        const double2 c = C[i];
        if (stage == 1) {
            Cacc[i] = k;
            Cstage[i] = cadd(c, cscale(k, 0.5 * dt));
        } else if (stage == 2) {
            Cacc[i] = cadd(Cacc[i], cscale(k, 2.0));
            Cstage[i] = cadd(c, cscale(k, 0.5 * dt));
        } else if (stage == 3) {
            Cacc[i] = cadd(Cacc[i], cscale(k, 2.0));
            Cstage[i] = cadd(c, cscale(k, dt));
        } else {
            const double2 cn = cadd(c, cscale(cadd(Cacc[i], k), dt / 6.0));
            C[i] = cn;
            bad |= !(isfinite(cn.x) && isfinite(cn.y));
            if (i < N) {
                r[i] = r_new[i];
                R[i] = R_new[i];
            }
        }
    }
    if (bad) {
        atomicOr(&flags[kFlagNonfinite], 1);
        atomicOr(&flags[kFlagHalt], 1);
    }
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

void launch_assemble(const Dims &d, const Bufs &b, int parity, bool initial, hipStream_t s) {
    const int Np = padded(d.N);
    const size_t tot = (size_t)Np * Np;
    const int cur = parity, nxt = initial ? parity : 1 - parity;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, b.S1, b.S2, b.E1a, b.E1b,
                       b.E2a, b.E2b, b.Wc, b.Smat[cur], b.Kmat[cur], b.r, b.R, b.r_new, b.R_new, d.mp, d.N, Np,
                       d.eps, initial ? 1 : 0, b.Smat[nxt], b.Kminus, b.Kmat[nxt], b.Lmid, b.L[nxt], b.Kmid,
                       b.flags);
}

void launch_cholesky(const Dims &d, const Bufs &b, double2 *A0, double2 *A1, int count, hipStream_t s) {
    const int Np = padded(d.N);
    for (int kb = 0; kb < Np; kb += NB) {
        const int below = Np - kb - NB;
        const int gx = below > 0 ? below / 64 : 1;
        hipLaunchKernelGGL(k_chol_panel, dim3(gx, count), dim3(64), 0, s, A0, A1, Np, kb, b.chol_diag, b.flags);
        if (below > 0) {
            const int mt = below / 32;
            hipLaunchKernelGGL(k_chol_update, dim3(mt * (mt + 1) / 2, count), dim3(64), 0, s, A0, A1, Np, kb,
                               b.flags);
        }
    }
    hipLaunchKernelGGL(k_chol_flush, dim3(1, count), dim3(64), 0, s, A0, A1, Np, Np - NB, b.chol_diag, b.flags);
}

void launch_rk4(const Dims &d, const Bufs &b, int parity, hipStream_t s) {
    const int Np = padded(d.N);
    const int cur = parity, nxt = 1 - parity;
    const double2 *Ks[4] = {b.Kmat[cur], b.Kmid, b.Kmid, b.Kminus};
    const double2 *Ls[4] = {b.L[cur], b.Lmid, b.Lmid, b.L[nxt]};
    const size_t lds = Np <= kSolveLdsMax ? sizeof(double2) * Np : 0;
    for (int st = 1; st <= 4; ++st) {
        const double2 *v = (st == 1) ? b.C : b.Cstage;
        hipLaunchKernelGGL(k_matvec, dim3(Np / 4), dim3(256), 0, s, Ks[st - 1], v, b.y, Np, b.flags);
        hipLaunchKernelGGL(k_rk_stage, dim3(1), dim3(1024), lds, s, Ls[st - 1], b.y, st, d.dt, d.N, Np, b.C,
                           b.Cacc, b.Cstage, b.r, b.R, b.r_new, b.R_new, b.flags);
    }
}

void launch_solve_initial(const Dims &d, const Bufs &b, int parity, double2 *rhs, hipStream_t s) {
    const int Np = padded(d.N);
    const size_t lds = Np <= kSolveLdsMax ? sizeof(double2) * Np : 0;
    hipLaunchKernelGGL(k_rk_stage, dim3(1), dim3(1024), lds, s, b.L[parity], rhs, 0, d.dt, d.N, Np, b.C, b.Cacc,
                       b.Cstage, b.r, b.R, b.r_new, b.R_new, b.flags);
}

void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

}  // namespace icwf
