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
// 64-wide panels.  Each k_chol_panel work-group eliminates, column by column,
// the 96 x 64 slab of the diagonal block and 32 of the rows below it, held
// in registers (lane = column, wave = 8 rows; the pivot column through LDS,
// one barrier per column); every work-group factors the diagonal block
// itself, so the panel needs no communication between work-groups.
// k_chol_update subtracts L21 L21^H from the trailing lower triangle on FP64
// matrix cores.  A pivot that is not positive raises the solve flag.
//
// RK4 (classical, S and K linear in time between the step ends, so the
// midpoint is their average).  Each stage is a matvec K v over many
// work-groups and two launches over the 64-row blocks of the factor.
// k_rk_fwd: a work-group solves L y = K v for its block after the blocks
// above it are done (it waits on their flags and subtracts their
// contributions as they arrive), then applies the inverse of its diagonal
// block (from k_tri_inv, computed beside the two-body contraction).
// k_rk_bwd: the same for L^H x = y from the bottom up, then the stage update
// k = -i x of its rows.  Work-groups take blocks in ticket order, so a
// work-group only ever waits on work-groups that are already running, and
// every wait is bounded.
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
                           int part, double2 *__restrict__ Snext, double2 *__restrict__ Kminus,
                           double2 *__restrict__ Knext, double2 *__restrict__ Amid, double2 *__restrict__ Anext,
                           double2 *__restrict__ Kmid, const int32_t *__restrict__ flags, const long long *__restrict__ zoff, const ModelParams *__restrict__ mpd) {
    const long long zo_ = batch_offset(zoff);
    S1 = zshift(S1, zo_);
    S2 = zshift(S2, zo_);
    E1a = zshift(E1a, zo_);
    E1b = zshift(E1b, zo_);
    E2a = zshift(E2a, zo_);
    E2b = zshift(E2b, zo_);
    Wc = zshift(Wc, zo_);
    Scur = zshift(Scur, zo_);
    Kcur = zshift(Kcur, zo_);
    r = zshift(r, zo_);
    R = zshift(R, zo_);
    r_new = zshift(r_new, zo_);
    R_new = zshift(R_new, zo_);
    Snext = zshift(Snext, zo_);
    Kminus = zshift(Kminus, zo_);
    Knext = zshift(Knext, zo_);
    Amid = zshift(Amid, zo_);
    Anext = zshift(Anext, zo_);
    Kmid = zshift(Kmid, zo_);
    flags = zshift(flags, zo_);
    if (zoff) mp = *zshift(mpd, zo_);

    if (flags[kFlagHalt]) return;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Np * Np) return;
    const int b = (int)(idx / Np), a = (int)(idx - (size_t)b * Np);
    const double2 s1 = S1[idx], s2 = S2[idx];
    const double2 S = cmul(s1, s2);
    const double reg = (a == b) ? eps : 0.0;
    if (part & kAssembleS) {
        Snext[idx] = S;
        Anext[idx] = make_double2(S.x + reg, S.y);
        if (part == kAssembleS) {
            const double2 sc = Scur[idx];
            Amid[idx] = make_double2(0.5 * (sc.x + S.x) + reg, 0.5 * (sc.y + S.y));
        }
    }
    if (!(part & kAssembleK)) return;
    const double2 w = (b <= a) ? Wc[idx] : cconj(Wc[(size_t)a * Np + b]);
    double ca = 0.0, cn = 0.0;
    if (a < N) {
        ca = model_v1(mp, r[a]) + model_v2(mp, R[a]);
        cn = model_v1(mp, r_new[a]) + model_v2(mp, R_new[a]);
    }
    if (part != kAssembleKnext) {
        const double2 km = csub(csub(csub(w, cmul(E1a[idx], s2)), cmul(s1, E2a[idx])), cscale(S, ca));
        if (part == kAssembleInitial) {
            // start of the run: K_0 = K(psi_0, x_0) -> the slot of parity 0
            Knext[idx] = km;
            return;
        }
        Kminus[idx] = km;
        const double2 kc = Kcur[idx];
        Kmid[idx] = make_double2(0.5 * (kc.x + km.x), 0.5 * (kc.y + km.y));
    }
    if (part != kAssembleKminus)
        Knext[idx] = csub(csub(csub(w, cmul(E1b[idx], s2)), cmul(s1, E2b[idx])), cscale(S, cn));
}

// ------------------------------------------------------------------ Cholesky
constexpr int NB = kCholNb;   // 64

__device__ inline void raise_solve(int32_t *flags) {
    atomicOr(&flags[kFlagSolve], 1);
    atomicOr(&flags[kFlagHalt], 1);
}

// Packed lower-triangular tile of NB x NB entries in LDS, column-major:
// entry (row k, column j), k >= j, at colofs(j) + k - j.
__host__ __device__ constexpr int colofs(int j) { return j * NB - j * (j - 1) / 2; }
// Row-major packing: entry (row j, column i), i <= j, at rowofs(j) + i.
__host__ __device__ constexpr int rowofs(int j) { return j * (j + 1) / 2; }
constexpr int kPacked = NB * (NB + 1) / 2;

// Broadcast lane `src` (wave-uniform) of a double to the whole wave.
__device__ inline double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// The panel: the 64 x 64 diagonal block stacked on this work-group's 32 rows
// below it (a 96 x 64 slab), eliminated column by column (right-looking):
// step j takes the pivot d = sqrt(a_jj) and subtracts
// l_rj conj(l_cj) = a_rj conj(a_cj) / d^2 from every later column c; column j
// below the pivot is scaled by 1/d once, after the last step (its entries do
// not change after step j, and the updates use the unscaled values).  On the
// diagonal rows this is the Cholesky factor L11; on the rows below it is
// x L11^H = a.
// 768 threads: wave g owns slab rows 8 g .. 8 g + 7 (g < 8: diagonal-block
// rows; g >= 8: 8 of the rows below), lane c owns column c; 8 entries per
// thread in registers with static indices.  At step j a wave takes its rows'
// column-j entries from lane j by readlane; the column-j entries of the
// diagonal rows (the pivot and every lane's a_cj) come through LDS, written by
// lane j of the diagonal waves as soon as their step j - 1 update is done, so
// one barrier per step publishes them.  The update runs on every entry of a
// lane's column, branch-free: entries above the diagonal of the block are
// updated too but never read (the factor is written from the lower part only).
//
// The factored diagonal block goes to a scratch tile, not into A: other
// work-groups of the same launch may still be reading the unfactored block.
// Work-group 0 of the next launch (or k_chol_flush after the last panel) copies
// it into place.  32 rows below per work-group rather than 64 where the
// launch's work-groups fit the CU slots left to the factorisations (the first
// panel at N = 1024 takes 60 of the 64 the FP64 contraction leaves free):
// a quarter fewer waves per SIMD issue each column's updates (the
// factorisation stream at N = 1024: 3.87 -> 3.69 ms stretched); else 64, in
// one round of work-groups rather than two.
constexpr int kPanelRows = 8;                   // slab rows per wave
constexpr int kPanelDiagWaves = NB / kPanelRows;
constexpr int panel_threads(int below) { return 64 * (NB + below) / kPanelRows; }

template <int BELOW>   // rows below the diagonal block per work-group: 32 or 64
__global__ void __launch_bounds__(panel_threads(BELOW)) k_chol_panel(double2 *A0, double2 *A1, int Np, int kb,
                                                              double2 *__restrict__ diag,
                                                              int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    A0 = zshift(A0, zo_);
    A1 = zshift(A1, zo_);
    diag = zshift(diag, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    // the panel is a latency chain that shares compute units with the
    // contraction on the other stream: its waves take the issue slots first
    __builtin_amdgcn_s_setprio(3);
    __shared__ double2 lcol[2][NB];      // column j over the diagonal rows, unscaled, alternating with j
    __shared__ double dpiv[NB], dinvs[NB];
    double2 *A = blockIdx.y ? A1 : A0;
    double2 *D = diag + (size_t)blockIdx.y * NB * NB;
    const int t = threadIdx.x, c = t & 63, g = t >> 6;
    if (blockIdx.x == 0 && kb > 0) {
        const int pb = kb - NB;
        for (int e = t; e < NB * NB; e += panel_threads(BELOW)) {
            const int rr = e / NB, cc = e % NB;
            if (cc <= rr) A[(size_t)(pb + rr) * Np + pb + cc] = D[e];
        }
    }
    const bool below = kb + NB < Np;
    const bool diagw = g < kPanelDiagWaves;
    const bool mine = diagw || below;                 // rows below exist for this wave
    const int srow = kPanelRows * g;                  // first slab row of this wave
    const int grow = diagw ? kb + srow : kb + NB + blockIdx.x * BELOW + kPanelRows * (g - kPanelDiagWaves);
    double2 a[kPanelRows];
#pragma unroll
    for (int v = 0; v < kPanelRows; ++v)
        a[v] = mine ? A[(size_t)(grow + v) * Np + kb + c] : make_double2(0.0, 0.0);
    if (c == 0 && diagw) {
#pragma unroll
        for (int v = 0; v < kPanelRows; ++v) lcol[0][srow + v] = a[v];
    }
    __syncthreads();
    bool bad = false;
#pragma unroll 1
    for (int j = 0; j < NB; ++j) {
        const double2 *lj = lcol[j & 1];
        double piv = lj[j].x;
        const double2 lcj = lj[c];
        double2 lr[kPanelRows];
#pragma unroll
        for (int v = 0; v < kPanelRows; ++v) lr[v] = make_double2(bcast(a[v].x, j), bcast(a[v].y, j));
        if (!(piv > 0.0)) {
            bad = true;
            piv = 1.0;
        }
        // 1/sqrt(piv) from the hardware estimate and two Newton steps
        // y <- y (3 - piv y^2) / 2 (each squares the relative error), then
        // sqrt(piv) = piv y: a few FP64 operations instead of the correctly
        // rounded sqrt and division sequences on the panel's serial chain
        double dinv = __builtin_amdgcn_rsq(piv);
        dinv = dinv * fma(-0.5 * piv * dinv, dinv, 1.5);
        dinv = dinv * fma(-0.5 * piv * dinv, dinv, 1.5);
        const double d = piv * dinv;
        if (c > j) {
            const double2 lc = cscale(cconj(lcj), dinv * dinv);
#pragma unroll
            for (int v = 0; v < kPanelRows; ++v) a[v] = csub(a[v], cmul(lr[v], lc));
            if (c == j + 1 && diagw) {
                double2 *ln = lcol[(j + 1) & 1];
#pragma unroll
                for (int v = 0; v < kPanelRows; ++v) ln[srow + v] = a[v];
            }
        } else if (t == j) {
            dpiv[j] = d;
            dinvs[j] = dinv;
        }
        __syncthreads();
    }
    if (bad && t == 0 && blockIdx.x == 0) raise_solve(flags);
    const double sc = dinvs[c];
#pragma unroll
    for (int v = 0; v < kPanelRows; ++v) a[v] = cscale(a[v], sc);
    if (diagw) {
        if (blockIdx.x == 0) {
#pragma unroll
            for (int v = 0; v < kPanelRows; ++v) {
                const int r = srow + v;
                if (r > c) D[r * NB + c] = a[v];
                else if (r == c) D[r * NB + c] = make_double2(dpiv[c], 0.0);
            }
        }
    } else if (below) {
#pragma unroll
        for (int v = 0; v < kPanelRows; ++v) A[(size_t)(grow + v) * Np + kb + c] = a[v];
    }
}

__global__ void __launch_bounds__(256) k_chol_flush(double2 *A0, double2 *A1, int Np, int kb,
                                                    const double2 *__restrict__ diag,
                                                    const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    A0 = zshift(A0, zo_);
    A1 = zshift(A1, zo_);
    diag = zshift(diag, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    double2 *A = blockIdx.y ? A1 : A0;
    const double2 *D = diag + (size_t)blockIdx.y * NB * NB;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int rr = e / NB, cc = e % NB;
        if (cc <= rr) A[(size_t)(kb + rr) * Np + kb + cc] = D[e];
    }
}

// Trailing update A[i][k] -= sum_j L[i][j] conj(L[k][j]) over the lower
// triangle i >= k of rows/cols kb+NB .. Np-1, j over the panel; one
// work-group per 32 x 32 tile, wave w on its 16 x 16 fragment (w / 2, w % 2),
// so a tile's 64-deep reduction runs on four matrix-core streams at once.
__global__ void __launch_bounds__(256) k_chol_update(double2 *A0, double2 *A1, int Np, int kb,
                                                     const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    A0 = zshift(A0, zo_);
    A1 = zshift(A1, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    double2 *A = blockIdx.y ? A1 : A0;
    const int t = blockIdx.x;
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tk = t - ti * (ti + 1) / 2;
    const int base = kb + NB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int f = wave >> 1, g = wave & 1;
    const int i0 = base + 32 * ti + 16 * f, k0 = base + 32 * tk + 16 * g;
    const int row = lane & 15, quarter = lane >> 4;
    const int q = NB / 4;
    dbl4 re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
    const double2 *xp = A + (size_t)(i0 + row) * Np + kb + quarter * q;
    const double2 *yp = A + (size_t)(k0 + row) * Np + kb + quarter * q;
    for (int s = 0; s < q; ++s) {
        const double2 xv = xp[s], yv = yp[s];
        // x conj(y) = (xr yr + xi yi) + i (xi yr - xr yi)
        re = mfma(xv.x, yv.x, re);
        re = mfma(xv.y, yv.y, re);
        im = mfma(xv.y, yv.x, im);
        im = mfma(-xv.x, yv.y, im);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ii = i0 + mfma_row_f64(lane, v);
        const int kk = k0 + row;
        double2 *p = A + (size_t)ii * Np + kk;
        const double2 o = *p;
        *p = make_double2(o.x - re[v], o.y - im[v]);
    }
}

// Inverse of each 64 x 64 diagonal block of a lower Cholesky factor,
// X_B = L_BB^-1 (lower triangular), by block recursion:
//     [[A, 0], [C, D]]^-1 = [[A^-1, 0], [-D^-1 C A^-1, D^-1]].
// The four 16 x 16 diagonal blocks are inverted by the four waves at once
// (lane c of wave w substitutes column c of its block in registers:
// x_rc = (delta_rc - sum_{k<r} L_rk x_kc) / L_rr); the off-diagonal blocks of
// the two 32 x 32 inverses, then the one of the 64 x 64 inverse, are the
// products -D^-1 (C A^-1).  One work-group per block, a handful of barriers.
// The stage solves apply X_B and X_B^H as matrix-vector products instead of a
// 64-step substitution on their critical path.  Output: X[(B 64 + r) 64 + c].
__global__ void __launch_bounds__(256) k_tri_inv(const double2 *__restrict__ A0, const double2 *__restrict__ A1,
                                                 double2 *__restrict__ X0, double2 *__restrict__ X1,
                                                 double2 *__restrict__ F0, double2 *__restrict__ F1, int Np,
                                                 const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    A0 = zshift(A0, zo_);
    A1 = zshift(A1, zo_);
    X0 = zshift(X0, zo_);
    X1 = zshift(X1, zo_);
    F0 = zshift(F0, zo_);
    F1 = zshift(F1, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    // 66.5 KB of LDS: fits beside a two-body contraction work-group on one CU
    __shared__ double2 sX[NB][NB + 1];        // the inverse (lower; zero above)
    const double2 *A = blockIdx.y ? A1 : A0;
    double2 *X = blockIdx.y ? X1 : X0;
    double2 *F = blockIdx.y ? F1 : F0;        // the same blocks in a full Np x Np inverse, or null
    const int r0 = blockIdx.x * NB;
    const double2 *Lb = A + (size_t)r0 * Np + r0;   // L_BB(r, k) = Lb[r Np + k]
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int e = t; e < NB * (NB + 1); e += 256) sX[e / (NB + 1)][e % (NB + 1)] = make_double2(0.0, 0.0);
    __syncthreads();
    // 16 x 16 diagonal blocks (their entries are the same for every lane: cached loads)
    if (lane < 16) {
        const int c = lane, o = 16 * wave;
        const double2 *Ld = Lb + (size_t)o * Np + o;
        double2 x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double2 acc = make_double2(r == c ? 1.0 : 0.0, 0.0);
#pragma unroll
            for (int k = 0; k < r; ++k) acc = csub(acc, cmul(Ld[(size_t)r * Np + k], x[k]));
            x[r] = cscale(acc, 1.0 / Ld[(size_t)r * Np + r].x);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) sX[o + r][o + c] = x[r];
    }
    __syncthreads();
    // level 1: blocks (1, 0) and (3, 2) of 16: T = L_ba X_aa into sX, then -X_bb T
    {
        const int p = t >> 7, u = t & 127;            // pair p, 128 threads per pair, 2 outputs each
        const int a = 2 * p, bb = 2 * p + 1;
        double2 o2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = u + 128 * h, r = e >> 4, c = e & 15;
            double2 acc = make_double2(0.0, 0.0);
            for (int k = c; k < 16; ++k)
                acc = cadd(acc, cmul(Lb[(size_t)(16 * bb + r) * Np + 16 * a + k], sX[16 * a + k][16 * a + c]));
            o2[h] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = u + 128 * h, r = e >> 4, c = e & 15;
            sX[16 * bb + r][16 * a + c] = o2[h];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = u + 128 * h, r = e >> 4, c = e & 15;
            double2 acc = make_double2(0.0, 0.0);
            for (int k = 0; k <= r; ++k) acc = cadd(acc, cmul(sX[16 * bb + r][16 * bb + k], sX[16 * bb + k][16 * a + c]));
            o2[h] = make_double2(-acc.x, -acc.y);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = u + 128 * h, r = e >> 4, c = e & 15;
            sX[16 * bb + r][16 * a + c] = o2[h];
        }
        __syncthreads();
    }
    // level 2: block (1, 0) of 32: T = L_BA X_AA, then -X_BB T (4 outputs per thread)
    {
        double2 o4[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int e = t + 256 * h, r = e >> 5, c = e & 31;
            double2 acc = make_double2(0.0, 0.0);
            for (int k = c; k < 32; ++k) acc = cadd(acc, cmul(Lb[(size_t)(32 + r) * Np + k], sX[k][c]));
            o4[h] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int e = t + 256 * h, r = e >> 5, c = e & 31;
            sX[32 + r][c] = o4[h];
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int e = t + 256 * h, r = e >> 5, c = e & 31;
            double2 acc = make_double2(0.0, 0.0);
            for (int k = 0; k <= r; ++k) acc = cadd(acc, cmul(sX[32 + r][32 + k], sX[32 + k][c]));
            o4[h] = make_double2(-acc.x, -acc.y);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int e = t + 256 * h, r = e >> 5, c = e & 31;
            sX[32 + r][c] = o4[h];
        }
        __syncthreads();
    }
    for (int e = t; e < NB * NB; e += 256) {
        const int rr = e / NB, cc = e % NB;
        X[(size_t)(r0 + rr) * NB + cc] = sX[rr][cc];
        if (F) F[(size_t)(r0 + rr) * Np + r0 + cc] = sX[rr][cc];
    }
}

// ------------------------------------------------------------------ explicit inverse of L
// Batched complex GEMM on 64 x 64 output tiles, O = alpha A B; 4 waves per
// tile, each on a 32 x 32 quarter as 2 x 2 MFMA fragments (rows i, columns j,
// reduction k), 16-wide k chunks of A and B staged through double-buffered
// LDS.  Batch entry z: factor f = z / npairs, pair p = z % npairs, operands
// at base[f] + p stride.
struct GemmBatch {
    const double2 *A[2], *B[2];
    double2 *O[2];
    long long stride;      // element offset between consecutive pairs (A, B and O alike)
    int lda, ldb, ldo;
    int M, N, K;           // output rows and columns, reduction length (multiples of 64)
    int npairs;
    double alpha;
    int lower_a, lower_b;  // A / B lower triangular: the reduction skips the chunks that are zero
};

constexpr int kGT = 64, kGKC = 16, kGLD = kGKC + 1;

__global__ void __launch_bounds__(256, 2) k_cgemm(GemmBatch g, const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    __shared__ double2 sA[2][kGT][kGLD];   // [i][k] of A
    __shared__ double2 sB[2][kGT][kGLD];   // [j][k] of B
    const int z = blockIdx.z, f = z / g.npairs, p = z - f * g.npairs;
    const size_t off = (size_t)p * g.stride;
    const double2 *__restrict__ A = (f ? g.A[1] : g.A[0]) + off;
    const double2 *__restrict__ B = (f ? g.B[1] : g.B[0]) + off;
    double2 *__restrict__ O = (f ? g.O[1] : g.O[0]) + off;
    const int nt = g.N / kGT;
    const int ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int i0 = ti * kGT, j0 = tj * kGT;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int row = lane & 15, quarter = lane >> 4;
    const int wi = 32 * (wave >> 1), wj = 32 * (wave & 1);
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            re[a][c] = dbl4{0, 0, 0, 0};
            im[a][c] = dbl4{0, 0, 0, 0};
        }
    // B lower triangular: B[k][j] = 0 for k < j, so the tile's columns
    // j >= j0 need k >= j0; A lower triangular: rows i < i0 + 64 need
    // k < i0 + 64.  Only exact zeros are skipped.
    const int kbeg = g.lower_b ? j0 : 0;
    const int kend = g.lower_a ? min(g.K, i0 + kGT) : g.K;
    const int nch = kend > kbeg ? (kend - kbeg) / kGKC : 0;
    // staging: element e = t + 256 m (m < 4); A as [i][k] (64 x 16), B as
    // [k][j] (16 x 64); held as plain doubles (an array of double2 would be
    // placed in scratch memory)
    double rax[4], ray[4], rbx[4], rby[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = t + 256 * m;
            const double2 va = A[(size_t)(i0 + (e >> 4)) * g.lda + k0 + (e & 15)];
            const double2 vb = B[(size_t)(k0 + (e >> 6)) * g.ldb + j0 + (e & 63)];
            rax[m] = va.x;
            ray[m] = va.y;
            rbx[m] = vb.x;
            rby[m] = vb.y;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int e = t + 256 * m;
            sA[buf][e >> 4][e & 15] = make_double2(rax[m], ray[m]);
            sB[buf][e & 63][e >> 6] = make_double2(rbx[m], rby[m]);
        }
    };
    if (nch > 0) {
        fetch(kbeg);
        stash(0);
    }
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) fetch(kbeg + (ch + 1) * kGKC);
#pragma unroll
        for (int s4 = 0; s4 < kGKC / 4; ++s4) {
            const int kk = 4 * s4 + quarter;
            double2 xv[2], yv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                xv[a] = sA[buf][wi + 16 * a + row][kk];
                yv[a] = sB[buf][wj + 16 * a + row][kk];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    // x y = (xr yr - xi yi) + i (xr yi + xi yr)
                    re[a][c] = mfma(xv[a].x, yv[c].x, re[a][c]);
                    re[a][c] = mfma(-xv[a].y, yv[c].y, re[a][c]);
                    im[a][c] = mfma(xv[a].x, yv[c].y, im[a][c]);
                    im[a][c] = mfma(xv[a].y, yv[c].x, im[a][c]);
                }
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wi + 16 * a + mfma_row_f64(lane, v);
                const int j = j0 + wj + 16 * c + row;
                const double2 o = make_double2(g.alpha * re[a][c][v], g.alpha * im[a][c][v]);
                O[(size_t)i * g.ldo + j] = o;
            }
}

// ------------------------------------------------------------------ RK4 stage solves
// Synchronisation words in the workspace (int32): [0, 64) forward block
// flags, [64, 128) backward block flags, [128] forward ticket, [129] backward
// ticket.  Each kernel clears the other kernel's words for its next launch.
constexpr int kMaxBlocks = 64;
constexpr int kSyncFwd = 0, kSyncBwd = 64, kSyncTicketF = 128, kSyncTicketB = 129;

__device__ inline int take_ticket(int32_t *ctr, int *slot) {
    if (threadIdx.x == 0) *slot = atomicAdd(ctr, 1);
    __syncthreads();
    return *slot;
}

// Wait (thread 0, bounded) for a block flag, then let every wave acquire it.
__device__ inline void wait_block(const int32_t *flag, int32_t *status) {
    if (threadIdx.x == 0) wait_flag(flag, status);
    __syncthreads();
    (void)__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void publish_block(int32_t *flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        set_flag(flag);
    }
}

// Parts of a matrix a matrix-vector product reads: all of it, the lower
// triangle with the diagonal, or the upper triangle with the diagonal.
enum MatPart : int { kPartAll = 0, kPartLower = 1, kPartUpper = 2 };

// Row-times-vector sums of the stage solves: one row per 256-thread
// work-group, wave w taking the 64-column chunks w, w + 4, ... (so that a
// triangular part spreads evenly), the four wave sums added in wave order
// (a fixed summation order).  Every thread returns the row's sum.
template <typename Term>
__device__ inline double2 row_sum_wg(int rowi, int Np, int part, Term term) {
    __shared__ double2 wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lo = part == kPartUpper ? (rowi & ~63) : 0, hi = part == kPartLower ? rowi + 1 : Np;
    double2 acc = make_double2(0, 0);
    for (int c = lo + 64 * wave + lane; c < hi; c += 256)
        if (part != kPartUpper || c >= rowi) acc = cadd(acc, term(c));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc.x += __shfl_xor(acc.x, off);
        acc.y += __shfl_xor(acc.y, off);
    }
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    return cadd(cadd(wsum[0], wsum[1]), cadd(wsum[2], wsum[3]));
}

// y = M v over the part of M (one row per work-group)
__global__ void __launch_bounds__(256) k_matvec(const double2 *__restrict__ M, const double2 *__restrict__ v,
                                                double2 *__restrict__ y, int Np, int part,
                                                const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    M = zshift(M, zo_);
    v = zshift(v, zo_);
    y = zshift(y, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    const int rowi = blockIdx.x;
    const double2 *m = M + (size_t)rowi * Np;
    const double2 acc = row_sum_wg(rowi, Np, part, [&](int c) { return cmul(m[c], v[c]); });
    if (threadIdx.x == 0) y[rowi] = acc;
}

// Forward stage kernel: y_B = L_BB^-1 (rhs_B - sum_{C<B} L_BC y_C), with
// L_BB^-1 from k_tri_inv.  256 threads; thread t: row i = t / 4 of the block,
// quarter q = t % 4 of the columns.  Everything that does not depend on the
// blocks above (the block's slices of L and of L_BB^-1) is loaded before the
// waits.
__global__ void __launch_bounds__(256) k_rk_fwd(const double2 *__restrict__ rhs, const double2 *__restrict__ L,
                                                const double2 *__restrict__ Linv, double2 *__restrict__ ybuf,
                                                int Np, int32_t *__restrict__ sync, int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    rhs = zshift(rhs, zo_);
    L = zshift(L, zo_);
    Linv = zshift(Linv, zo_);
    ybuf = zshift(ybuf, zo_);
    sync = zshift(sync, zo_);
    flags = zshift(flags, zo_);

    __shared__ double2 uvec[NB];
    __shared__ int slot;
    const int B = take_ticket(&sync[kSyncTicketF], &slot);
    if (B == 0) {
        for (int e = threadIdx.x; e < kMaxBlocks; e += 256) sync[kSyncBwd + e] = 0;
        if (threadIdx.x == 0) sync[kSyncTicketB] = 0;
    }
    const bool halted = flags[kFlagHalt] != 0;
    const int t = threadIdx.x, i = t >> 2, q = t & 3;
    const int r0 = B * NB;
    double2 iv[16];   // row i of L_BB^-1, columns 16 q ..
#pragma unroll
    for (int c = 0; c < 16; ++c) iv[c] = halted ? make_double2(0, 0) : Linv[(size_t)(r0 + i) * NB + 16 * q + c];
    // contributions of the blocks above, as they complete
    double2 part = make_double2(0, 0);
    for (int C = 0; C < B; ++C) {
        double2 lv[16];
        const double2 *lrow = L + (size_t)(r0 + i) * Np + C * NB + 16 * q;
#pragma unroll
        for (int c = 0; c < 16; ++c) lv[c] = halted ? make_double2(0, 0) : lrow[c];
        wait_block(&sync[kSyncFwd + C], flags);
        if (halted) continue;
        const double2 *yc = ybuf + C * NB + 16 * q;
#pragma unroll
        for (int c = 0; c < 16; ++c) part = cadd(part, cmul(lv[c], yc[c]));
    }
    part.x += __shfl_xor(part.x, 1);
    part.y += __shfl_xor(part.y, 1);
    part.x += __shfl_xor(part.x, 2);
    part.y += __shfl_xor(part.y, 2);
    if (q == 0) uvec[i] = halted ? make_double2(0, 0) : csub(rhs[r0 + i], part);
    __syncthreads();
    double2 y = make_double2(0, 0);
#pragma unroll
    for (int c = 0; c < 16; ++c) y = cadd(y, cmul(iv[c], uvec[16 * q + c]));
    y.x += __shfl_xor(y.x, 1);
    y.y += __shfl_xor(y.y, 1);
    y.x += __shfl_xor(y.x, 2);
    y.y += __shfl_xor(y.y, 2);
    if (!halted && q == 0) ybuf[r0 + i] = y;
    publish_block(&sync[kSyncFwd + B]);
}

// The RK4 stage update of row ii from its solve x = (S + eps I)^-1 K v:
// k = -i x; stage 0 stores the initial coefficients C = x.
__device__ inline void stage_update(int ii, double2 u, int stage, double dt, int N, double2 *__restrict__ C,
                                    double2 *__restrict__ Cacc, double2 *__restrict__ Cstage,
                                    double *__restrict__ r, double *__restrict__ R,
                                    const double *__restrict__ r_new, const double *__restrict__ R_new,
                                    int32_t *__restrict__ flags) {
    bool bad = false;
    if (stage == 0) {
        C[ii] = (ii < N) ? u : make_double2(0, 0);
        bad = !(isfinite(u.x) && isfinite(u.y));
    } else {
        const double2 k = make_double2(u.y, -u.x);   // -i x
        const double2 c = C[ii];
        if (stage == 1) {
            Cacc[ii] = k;
            Cstage[ii] = cadd(c, cscale(k, 0.5 * dt));
        } else if (stage == 2) {
            Cacc[ii] = cadd(Cacc[ii], cscale(k, 2.0));
            Cstage[ii] = cadd(c, cscale(k, 0.5 * dt));
        } else if (stage == 3) {
            Cacc[ii] = cadd(Cacc[ii], cscale(k, 2.0));
            Cstage[ii] = cadd(c, cscale(k, dt));
        } else {
            const double2 cn = cadd(c, cscale(cadd(Cacc[ii], k), dt / 6.0));
            C[ii] = cn;
            bad = !(isfinite(cn.x) && isfinite(cn.y));
            if (ii < N && r) {   // r == nullptr: Heun trajectories, positions set by the corrector
                r[ii] = r_new[ii];
                R[ii] = R_new[ii];
            }
        }
    }
    if (bad) {
        atomicOr(&flags[kFlagNonfinite], 1);
        atomicOr(&flags[kFlagHalt], 1);
    }
}

// Backward stage kernel: x_B = L_BB^-H (y_B - sum_{C>B} L_CB^H x_C), blocks
// from the bottom up; then the RK4 stage update of the block's rows.
// stage: 1..4; 0 = initial coefficients (C = x).
__global__ void __launch_bounds__(256) k_rk_bwd(const double2 *__restrict__ L, const double2 *__restrict__ Linv,
                                                const double2 *__restrict__ ybuf, double2 *__restrict__ xbuf, int Np,
                                                int nblk, int stage, double dt, int N, double2 *__restrict__ C,
                                                double2 *__restrict__ Cacc, double2 *__restrict__ Cstage,
                                                double *__restrict__ r, double *__restrict__ R,
                                                const double *__restrict__ r_new, const double *__restrict__ R_new,
                                                int32_t *__restrict__ sync, int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    L = zshift(L, zo_);
    Linv = zshift(Linv, zo_);
    ybuf = zshift(ybuf, zo_);
    xbuf = zshift(xbuf, zo_);
    C = zshift(C, zo_);
    Cacc = zshift(Cacc, zo_);
    Cstage = zshift(Cstage, zo_);
    r = zshift(r, zo_);
    R = zshift(R, zo_);
    r_new = zshift(r_new, zo_);
    R_new = zshift(R_new, zo_);
    sync = zshift(sync, zo_);
    flags = zshift(flags, zo_);

    __shared__ double2 uvec[NB];
    __shared__ int slot;
    const int ticket = take_ticket(&sync[kSyncTicketB], &slot);
    const int B = nblk - 1 - ticket;
    if (ticket == 0) {
        for (int e = threadIdx.x; e < kMaxBlocks; e += 256) sync[kSyncFwd + e] = 0;
        if (threadIdx.x == 0) sync[kSyncTicketF] = 0;
    }
    const bool halted = flags[kFlagHalt] != 0;
    const int t = threadIdx.x, i = t >> 2, q = t & 3;
    const int r0 = B * NB;
    double2 iv[16];   // column i of L_BB^-1, rows 16 q ..
#pragma unroll
    for (int c = 0; c < 16; ++c) iv[c] = halted ? make_double2(0, 0) : Linv[(size_t)(r0 + 16 * q + c) * NB + i];
    // contributions of the blocks below (already solved): sum_k conj(L[C64+k][B64+i]) x[C64+k]
    double2 part = make_double2(0, 0);
    for (int Cb = nblk - 1; Cb > B; --Cb) {
        double2 lv[16];
        const double2 *lcol = L + (size_t)(Cb * NB + 16 * q) * Np + r0 + i;
#pragma unroll
        for (int c = 0; c < 16; ++c) lv[c] = halted ? make_double2(0, 0) : lcol[(size_t)c * Np];
        wait_block(&sync[kSyncBwd + Cb], flags);
        if (halted) continue;
        const double2 *xc = xbuf + Cb * NB + 16 * q;
#pragma unroll
        for (int c = 0; c < 16; ++c) part = cadd(part, cmul(cconj(lv[c]), xc[c]));
    }
    part.x += __shfl_xor(part.x, 1);
    part.y += __shfl_xor(part.y, 1);
    part.x += __shfl_xor(part.x, 2);
    part.y += __shfl_xor(part.y, 2);
    if (q == 0) uvec[i] = halted ? make_double2(0, 0) : csub(ybuf[r0 + i], part);
    __syncthreads();
    double2 u = make_double2(0, 0);
#pragma unroll
    for (int c = 0; c < 16; ++c) u = cadd(u, cmul(cconj(iv[c]), uvec[16 * q + c]));
    u.x += __shfl_xor(u.x, 1);
    u.y += __shfl_xor(u.y, 1);
    u.x += __shfl_xor(u.x, 2);
    u.y += __shfl_xor(u.y, 2);
    if (!halted && q == 0) {
        xbuf[r0 + i] = u;
        stage_update(r0 + i, u, stage, dt, N, C, Cacc, Cstage, r, R, r_new, R_new, flags);
    }
    publish_block(&sync[kSyncBwd + B]);
}

// Stages through the explicit inverse of the factor, A^-1 = L^-H L^-1, with
// one step of iterative refinement: x0 = L^-H (L^-1 rhs) (two triangular
// k_matvec), res = rhs - A x0 (k_rk_resid, A formed from S as in the
// assembly), x = x0 + L^-H (L^-1 res) (k_matvec, then k_rk_apply with the
// stage update of the row).  The refinement brings the explicit inverse's
// error, of the order of cond(A) times its rounding, back to that of a
// solve with the factor.  One row per work-group.
__global__ void __launch_bounds__(256) k_rk_resid(const double2 *__restrict__ Sa, const double2 *__restrict__ Sb,
                                                  double eps, const double2 *__restrict__ x,
                                                  const double2 *__restrict__ rhs, double2 *__restrict__ res, int Np,
                                                  const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    Sa = zshift(Sa, zo_);
    Sb = zshift(Sb, zo_);
    x = zshift(x, zo_);
    rhs = zshift(rhs, zo_);
    res = zshift(res, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    const int rowi = blockIdx.x;
    const double2 *ma = Sa + (size_t)rowi * Np;
    const double2 *mb = Sb ? Sb + (size_t)rowi * Np : nullptr;
    const double2 acc = row_sum_wg(rowi, Np, kPartAll, [&](int c) {
        const double reg = (c == rowi) ? eps : 0.0;
        const double2 sa = ma[c];
        double2 a;
        if (mb) {                                    // midpoint: (S_a + S_b) / 2 + eps I
            const double2 sb = mb[c];
            a = make_double2(0.5 * (sa.x + sb.x) + reg, 0.5 * (sa.y + sb.y));
        } else {                                     // endpoint: S_a + eps I
            a = make_double2(sa.x + reg, sa.y);
        }
        return cmul(a, x[c]);
    });
    if (threadIdx.x == 0) res[rowi] = csub(rhs[rowi], acc);
}

__global__ void __launch_bounds__(256) k_rk_apply(const double2 *__restrict__ H, const double2 *__restrict__ z,
                                                  const double2 *__restrict__ x0, int Np, int stage, double dt, int N,
                                                  double2 *__restrict__ C, double2 *__restrict__ Cacc,
                                                  double2 *__restrict__ Cstage, double *__restrict__ r,
                                                  double *__restrict__ R, const double *__restrict__ r_new,
                                                  const double *__restrict__ R_new, int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    H = zshift(H, zo_);
    z = zshift(z, zo_);
    x0 = zshift(x0, zo_);
    C = zshift(C, zo_);
    Cacc = zshift(Cacc, zo_);
    Cstage = zshift(Cstage, zo_);
    r = zshift(r, zo_);
    R = zshift(R, zo_);
    r_new = zshift(r_new, zo_);
    R_new = zshift(R_new, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    const int rowi = blockIdx.x;
    const double2 *m = H + (size_t)rowi * Np;
    const double2 acc = row_sum_wg(rowi, Np, kPartUpper, [&](int c) { return cmul(m[c], z[c]); });   // (L^-H z)_rowi
    if (threadIdx.x == 0)
        stage_update(rowi, cadd(x0[rowi], acc), stage, dt, N, C, Cacc, Cstage, r, R, r_new, R_new, flags);
}

// H = F^H over the lower part of F (F = L^-1): 32 x 32 tiles through LDS,
// tile (bi, bj) of F with bi >= bj to tile (bj, bi) of H (the parts of F
// above and of H below the diagonal are neither read nor written).
__global__ void __launch_bounds__(256) k_conj_transpose(const double2 *__restrict__ F0, const double2 *__restrict__ F1,
                                                        double2 *__restrict__ H0, double2 *__restrict__ H1, int Np,
                                                        const int32_t *__restrict__ flags) {
    if (flags[kFlagHalt]) return;
    const int bi = blockIdx.x, bj = blockIdx.y;
    if (bi < bj) return;
    const double2 *F = blockIdx.z ? F1 : F0;
    double2 *H = blockIdx.z ? H1 : H0;
    __shared__ double2 tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows per pass
#pragma unroll
    for (int r = ty; r < 32; r += 8) tile[r][tx] = F[(size_t)(32 * bi + r) * Np + 32 * bj + tx];
    __syncthreads();
#pragma unroll
    for (int r = ty; r < 32; r += 8) H[(size_t)(32 * bj + r) * Np + 32 * bi + tx] = cconj(tile[tx][r]);
}

__global__ void k_set_table(long long *__restrict__ tab, BatchTable t, int n) {
    if ((int)threadIdx.x < n) tab[threadIdx.x] = t.off[threadIdx.x];
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v, const long long *__restrict__ zoff) {
    const long long zo_ = batch_offset(zoff);
    p = zshift(p, zo_);

    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

void launch_assemble(const Dims &d, const Bufs &b, int parity, AssemblePart part, hipStream_t s) {
    const int Np = padded(d.N);
    const size_t tot = (size_t)Np * Np;
    const bool initial = part == kAssembleInitial;
    const int cur = parity, nxt = initial ? parity : 1 - parity;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((tot + 255) / 256), 1, d.batch), dim3(256), 0, s, b.S1, b.S2,
                       b.E1a, b.E1b, b.E2a, b.E2b, b.Wc, b.Smat[cur], b.Kmat[cur], b.r, b.R, b.r_new, b.R_new, d.mp,
                       d.N, Np, d.eps, (int)part, b.Smat[nxt], b.Kminus, b.Kmat[nxt], b.Lmid, b.L[nxt], b.Kmid, b.flags,
                       d.zoff, d.mpd);
}

void launch_cholesky(const Dims &d, const Bufs &b, double2 *A0, double2 *A1, double2 *X0, double2 *X1, int count,
                     hipStream_t s, double2 *F0, double2 *F1, double2 *H0, double2 *H1, bool inverses) {
    const int Np = padded(d.N);
    // the CU slots the contraction leaves free (two work-groups per CU):
    // 32 rows below per panel work-group where the first launch fits them
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    const int free_slots = std::max(2 * ncu - d.wc_grid, 1);
    const bool narrow = (long long)count * d.batch * ((Np - NB) / 32) <= free_slots;
    for (int kb = 0; kb < Np; kb += NB) {
        const int below = Np - kb - NB;
        if (narrow) {
            const int gx = below > 0 ? below / 32 : 1;
            hipLaunchKernelGGL(k_chol_panel<32>, dim3(gx, count, d.batch), dim3(panel_threads(32)), 0, s, A0, A1, Np,
                               kb, b.chol_diag, b.flags, d.zoff);
        } else {
            const int gx = below > 0 ? below / 64 : 1;
            hipLaunchKernelGGL(k_chol_panel<64>, dim3(gx, count, d.batch), dim3(panel_threads(64)), 0, s, A0, A1, Np,
                               kb, b.chol_diag, b.flags, d.zoff);
        }
        if (below > 0) {
            const int mt = below / 32;
            hipLaunchKernelGGL(k_chol_update, dim3(mt * (mt + 1) / 2, count, d.batch), dim3(256), 0, s, A0, A1, Np, kb,
                               b.flags, d.zoff);
        }
    }
    hipLaunchKernelGGL(k_chol_flush, dim3(1, count, d.batch), dim3(256), 0, s, A0, A1, Np, Np - NB, b.chol_diag,
                       b.flags, d.zoff);
    hipLaunchKernelGGL(k_tri_inv, dim3(Np / NB, count, d.batch), dim3(256), 0, s, A0, A1, X0, X1, F0, F1, Np, b.flags,
                       d.zoff);
    if (F0 && inverses) launch_factor_inverses(d, b, A0, A1, count, s, F0, F1, H0, H1);
}

void launch_factor_inverses(const Dims &d, const Bufs &b, const double2 *A0, const double2 *A1, int count,
                            hipStream_t s, double2 *F0, double2 *F1, double2 *H0, double2 *H1) {
    const int Np = padded(d.N);
    double2 *Fs[2] = {F0, F1 ? F1 : F0};
    // X = L^-1 by block recursion, [[A, 0], [C, D]]^-1 = [[A', 0], [-D' C A', D']],
    // from the 64 x 64 diagonal inverses up: at block size h, the Np / (2 h) pairs
    // of every factor take T = C A' and then -D' T (X's upper triangle stays zero)
    const double2 *L2[2] = {A0, A1};
    for (int h = NB; h < Np; h *= 2) {
        GemmBatch g{};
        g.lda = g.ldb = g.ldo = Np;
        g.M = g.N = g.K = h;
        g.npairs = Np / (2 * h);
        g.stride = 2LL * h * (Np + 1);
        const dim3 grid((h / kGT) * (h / kGT), 1, count * g.npairs);
        for (int f = 0; f < 2; ++f) {                      // T = C A'
            g.A[f] = L2[f] + (size_t)h * Np;
            g.B[f] = Fs[f];
            g.O[f] = b.Tinv[f] + (size_t)h * Np;
        }
        g.alpha = 1.0;
        g.lower_a = 0;
        g.lower_b = 1;                                     // A' lower triangular
        hipLaunchKernelGGL(k_cgemm, grid, dim3(256), 0, s, g, b.flags);
        for (int f = 0; f < 2; ++f) {                      // X_DA = -D' T
            g.A[f] = Fs[f] + (size_t)h * Np + h;
            g.B[f] = b.Tinv[f] + (size_t)h * Np;
            g.O[f] = Fs[f] + (size_t)h * Np;
        }
        g.alpha = -1.0;
        g.lower_a = 1;                                     // D' lower triangular
        g.lower_b = 0;
        hipLaunchKernelGGL(k_cgemm, grid, dim3(256), 0, s, g, b.flags);
    }
    // L^-H for the stage solves
    hipLaunchKernelGGL(k_conj_transpose, dim3(Np / 32, Np / 32, count), dim3(256), 0, s, F0, F1 ? F1 : F0, H0,
                       H1 ? H1 : H0, Np, b.flags);
}

void launch_rk4(const Dims &d, const Bufs &b, int parity, hipStream_t s) {
    const int Np = padded(d.N), nblk = Np / NB;
    const int cur = parity, nxt = 1 - parity;
    const double2 *Ks[4] = {b.Kmat[cur], b.Kmid, b.Kmid, b.Kminus};
    const double2 *Ls[4] = {b.L[cur], b.Lmid, b.Lmid, b.L[nxt]};
    const double2 *Xs[4] = {b.Linv[cur], b.Linvmid, b.Linvmid, b.Linv[nxt]};
    const double2 *Fs[4] = {b.Finv[cur], b.Finvmid, b.Finvmid, b.Finv[nxt]};
    const double2 *Hs[4] = {b.Hinv[cur], b.Hinvmid, b.Hinvmid, b.Hinv[nxt]};
    // with Heun trajectories the last stage leaves x_k in place for the corrector
    double *cr = d.traj == 1 ? nullptr : b.r, *cR = d.traj == 1 ? nullptr : b.R;
    for (int st = 1; st <= 4; ++st) {
        const double2 *v = (st == 1) ? b.C : b.Cstage;
        hipLaunchKernelGGL(k_matvec, dim3(Np, 1, d.batch), dim3(256), 0, s, Ks[st - 1], v, b.rhs, Np,
                           (int)kPartAll, b.flags, d.zoff);
        if (d.sinv) {
            // A of the stage: S_k + eps I, the midpoint average + eps I (stages 2, 3), S_k+1 + eps I
            const double2 *Sa = st == 4 ? b.Smat[nxt] : b.Smat[cur];
            const double2 *Sb = (st == 2 || st == 3) ? b.Smat[nxt] : nullptr;
            hipLaunchKernelGGL(k_matvec, dim3(Np, 1, d.batch), dim3(256), 0, s, Fs[st - 1], b.rhs, b.zvec, Np,
                               (int)kPartLower, b.flags, d.zoff);
            hipLaunchKernelGGL(k_matvec, dim3(Np, 1, d.batch), dim3(256), 0, s, Hs[st - 1], b.zvec, b.y, Np,
                               (int)kPartUpper, b.flags, d.zoff);
            hipLaunchKernelGGL(k_rk_resid, dim3(Np, 1, d.batch), dim3(256), 0, s, Sa, Sb, d.eps, b.y, b.rhs, b.xsol,
                               Np, b.flags, d.zoff);
            hipLaunchKernelGGL(k_matvec, dim3(Np, 1, d.batch), dim3(256), 0, s, Fs[st - 1], b.xsol, b.zvec, Np,
                               (int)kPartLower, b.flags, d.zoff);
            hipLaunchKernelGGL(k_rk_apply, dim3(Np, 1, d.batch), dim3(256), 0, s, Hs[st - 1], b.zvec, b.y, Np, st,
                               d.dt, d.N, b.C, b.Cacc, b.Cstage, cr, cR, b.r_new, b.R_new, b.flags, d.zoff);
            continue;
        }
        hipLaunchKernelGGL(k_rk_fwd, dim3(nblk, 1, d.batch), dim3(256), 0, s, b.rhs, Ls[st - 1], Xs[st - 1], b.y, Np,
                           b.solve_sync, b.flags, d.zoff);
        hipLaunchKernelGGL(k_rk_bwd, dim3(nblk, 1, d.batch), dim3(256), 0, s, Ls[st - 1], Xs[st - 1], b.y, b.xsol, Np,
                           nblk, st, d.dt, d.N, b.C, b.Cacc, b.Cstage, cr, cR, b.r_new, b.R_new, b.solve_sync, b.flags,
                           d.zoff);
    }
}

void launch_solve_initial(const Dims &d, const Bufs &b, int parity, double2 *rhs, hipStream_t s) {
    const int Np = padded(d.N), nblk = Np / NB;
    hipLaunchKernelGGL(k_rk_fwd, dim3(nblk), dim3(256), 0, s, rhs, b.L[parity], b.Linv[parity], b.y, Np,
                       b.solve_sync, b.flags, nullptr);
    hipLaunchKernelGGL(k_rk_bwd, dim3(nblk), dim3(256), 0, s, b.L[parity], b.Linv[parity], b.y, b.xsol, Np, nblk, 0,
                       d.dt, d.N, b.C, b.Cacc, b.Cstage, b.r, b.R, b.r_new, b.R_new, b.solve_sync, b.flags, nullptr);
}

void launch_set_table(long long *tab, const BatchTable &t, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_table, dim3(1), dim3(kMaxBatch), 0, s, tab, t, n);
}

void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s, int batch, const long long *zoff) {
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256, 1, batch), dim3(256), 0, s, p, n, v, zoff);
}

}  // namespace icwf
