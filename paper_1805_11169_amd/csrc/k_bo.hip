// Born-Oppenheimer states on the GPU: the lowest eigenpairs of the clamped-
// nucleus electronic Hamiltonian h_e(R_j) = T_spec + diag(W(r_i, R_j)) for a
// list of R_j (the basis of the paper's BO populations and decoherence
// indicator, and of its initial state, the first excited BO state).
//
// One work-group per R_j runs block LOBPCG (Knyazev 2001) to the end in one
// launch:
//   * h_e is applied through the spectral kinetic operator, two real vectors
//     per complex transform (T is real and even in k, so T(u + i v) =
//     T u + i T v): a radix-2 transform in LDS, decimation in time from
//     bit-reversed input to natural order forward, the multiplier k^2/2m in
//     natural order, decimation in frequency back to bit-reversed order, then
//     + W(r_i, R_j) u_i;
//   * the preconditioner is (T_spec + c)^-1, the same transforms with the
//     multiplier 1/(k^2/2m + c), c = max(1, max W - min W) on the grid;
//   * each iteration orthonormalises [X, P(residuals), previous directions]
//     by classical Gram-Schmidt run twice (columns that lose all but 1e-10 of
//     their norm are dropped), applies h_e to the whole basis afresh, forms
//     the projected matrix and diagonalises it by cyclic Jacobi (parallel
//     round-robin ordering, rotations of Golub and Van Loan's symmetric 2 x 2
//     Schur form), then takes the m lowest Ritz pairs as the new block, the
//     non-X part of their coefficients as the new directions, and the
//     residuals h_e x - theta x;
//   * it stops when every wanted residual norm is at most tol.
// Vectors live in a per-R_j slice of the caller's workspace (L2-resident
// during the work-group's life); the transform buffer, the projected matrix
// and its rotations live in LDS.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/icwf_bo.h"
#include "icwf_plan.hpp"

namespace icwf {

namespace {

constexpr int kBoThreads = 256;
constexpr int kBoWaves = kBoThreads / 64;
constexpr int kBoMaxBlock = 12;              // n_states + guard vectors
constexpr int kBoMaxZ = 3 * kBoMaxBlock;     // columns of the Rayleigh-Ritz basis
constexpr int kChunk = 8;                    // dot products reduced together

struct BoArgs {
    int n, m, nwant, max_iter;
    double tol, r_min, h;
    ModelParams mp;
    const double *Rv;        // [nv]
    const double *kin;       // [n] k^2 / (2 m_r), FFT order
    const double2 *tw;       // [n / 2] exp(-2 pi i k / n)
    double *ws;              // per-value slices of ws_stride doubles
    size_t ws_stride;
    double *states;          // [nv][nwant][n] (grid-normalised)
    double *energies;        // [nv][nwant]
    int32_t *iters;          // [nv]
    double *resid;           // [nv]
    int32_t *flags;          // kFlagNonfinite on a non-finite potential
};

// Doubles of one R_j's slice: V, Z, HZ (kBoMaxZ columns each), X, P, Wr
// (kBoMaxBlock columns each).
inline size_t bo_stride(int n) { return (size_t)n * (1 + 2 * kBoMaxZ + 3 * kBoMaxBlock); }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sums cnt (<= kChunk) per-thread values over the work-group into out[0..cnt)
// (LDS), in a fixed order.
__device__ inline void block_sums(const double (&v)[kChunk], int cnt, double *red, double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
        if (c < cnt) {
            const double s = wave_sum(v[c]);
            if (lane == 0) red[wave * kChunk + c] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < cnt) {
        const int c = threadIdx.x;
        out[c] = ((red[c] + red[kChunk + c]) + red[2 * kChunk + c]) + red[3 * kChunk + c];
    }
    __syncthreads();
}

__device__ inline double block_sum1(double v, double *red, double *out) {
    double a[kChunk] = {v};
    block_sums(a, 1, red, out);
    return out[0];
}

// T or (T + c)^-1 applied to the pair (u, v) (v may be null), out to (ou, ov);
// with add_v the potential term V u is added (h_e).  fb: n complex in LDS.
template <int LOG2N>
__device__ void spectral_pair(const BoArgs &A, const double *u, const double *v, double *ou, double *ov,
                              const double *V, bool hamiltonian, double c, double2 *fb) {
    constexpr int n = 1 << LOG2N;
    const int tid = threadIdx.x;
    for (int e = tid; e < n; e += kBoThreads) {
        const int br = (int)(__brev((unsigned)e) >> (32 - LOG2N));
        fb[br] = make_double2(u[e], v ? v[e] : 0.0);
    }
    __syncthreads();
    // forward transform: decimation in time, bit-reversed in, natural out
#pragma unroll 1
    for (int s = 1; s <= LOG2N; ++s) {
        const int half = 1 << (s - 1), tstr = n >> s;
        for (int b = tid; b < n / 2; b += kBoThreads) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
            const double2 w = A.tw[pos * tstr];
            const double2 x0 = fb[i0], x1 = cmul(fb[i1], w);
            fb[i0] = cadd(x0, x1);
            fb[i1] = csub(x0, x1);
        }
        __syncthreads();
    }
    for (int k = tid; k < n; k += kBoThreads) {
        const double mult = hamiltonian ? A.kin[k] : 1.0 / (A.kin[k] + c);
        fb[k] = cscale(fb[k], mult);
    }
    __syncthreads();
    // inverse transform: decimation in frequency, natural in, bit-reversed out
#pragma unroll 1
    for (int s = LOG2N; s >= 1; --s) {
        const int half = 1 << (s - 1), tstr = n >> s;
        for (int b = tid; b < n / 2; b += kBoThreads) {
            const int pos = b & (half - 1);
            const int i0 = ((b >> (s - 1)) << s) + pos, i1 = i0 + half;
            const double2 w = cconj(A.tw[pos * tstr]);
            const double2 x0 = fb[i0], x1 = fb[i1];
            fb[i0] = cadd(x0, x1);
            fb[i1] = cmul(csub(x0, x1), w);
        }
        __syncthreads();
    }
    const double inv = 1.0 / n;
    for (int e = tid; e < n; e += kBoThreads) {
        const double2 y = fb[__brev((unsigned)e) >> (32 - LOG2N)];
        double yu = y.x * inv, yv = y.y * inv;
        if (hamiltonian) {
            yu += V[e] * u[e];
            if (v) yv += V[e] * v[e];
        }
        ou[e] = yu;
        if (v) ov[e] = yv;
    }
    __syncthreads();
}

// Appends candidate `src` to the orthonormal columns Z[0..cnt) by classical
// Gram-Schmidt twice; returns the new count (cnt + 1, or cnt if the
// candidate was (numerically) in their span).
template <int LOG2N>
__device__ int append_orthonormal(double *Z, int cnt, const double *src, double *red, double *dots) {
    constexpr int n = 1 << LOG2N;
    constexpr int per = n / kBoThreads > 0 ? n / kBoThreads : 1;
    const int tid = threadIdx.x;
    double *z = Z + (size_t)cnt * n;
    for (int e = tid; e < n; e += kBoThreads) z[e] = src[e];
    __syncthreads();
    double acc = 0.0;
    for (int e = tid; e < n; e += kBoThreads) acc += z[e] * z[e];
    const double n0 = sqrt(block_sum1(acc, red, dots + kBoMaxZ));
    if (!(n0 > 0.0) || !isfinite(n0)) return cnt;
    for (int pass = 0; pass < 2; ++pass) {
        for (int c0 = 0; c0 < cnt; c0 += kChunk) {
            const int cc = min(kChunk, cnt - c0);
            double part[kChunk] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int e = tid; e < n; e += kBoThreads) {
                const double ze = z[e];
#pragma unroll
                for (int q = 0; q < kChunk; ++q)
                    if (q < cc) part[q] += Z[(size_t)(c0 + q) * n + e] * ze;
            }
            block_sums(part, cc, red, dots + c0);
        }
        for (int e = tid; e < n; e += kBoThreads) {
            double ze = z[e];
            for (int i = 0; i < cnt; ++i) ze -= dots[i] * Z[(size_t)i * n + e];
            z[e] = ze;
        }
        __syncthreads();
    }
    (void)per;
    acc = 0.0;
    for (int e = tid; e < n; e += kBoThreads) acc += z[e] * z[e];
    const double n1 = sqrt(block_sum1(acc, red, dots + kBoMaxZ));
    if (!(n1 > 1e-10 * n0) || !isfinite(n1)) return cnt;
    const double inv = 1.0 / n1;
    for (int e = tid; e < n; e += kBoThreads) z[e] *= inv;
    __syncthreads();
    return cnt + 1;
}

// Eigen-decomposition of the symmetric k x k matrix G (LDS, row-major, k <=
// kBoMaxZ) by cyclic Jacobi: G -> diag(theta) ascending, Y the eigenvectors
// (columns).  Round-robin ordering: in each of K - 1 rounds (K = k rounded up
// to even) the K / 2 disjoint pairs rotate at once; player K - 1 stays, the
// others turn.
__device__ void jacobi(double *G, double *Y, int k, double *theta, double *red, double *scratch) {
    const int tid = threadIdx.x;
    __shared__ double cs[kBoMaxZ / 2], sn[kBoMaxZ / 2];
    __shared__ int pp[kBoMaxZ / 2], qq[kBoMaxZ / 2];
    for (int idx = tid; idx < k * k; idx += kBoThreads) Y[idx] = (idx / k == idx % k) ? 1.0 : 0.0;
    __syncthreads();
    const int K = (k + 1) & ~1, np = K / 2;
    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int idx = tid; idx < k * k; idx += kBoThreads) {
            const double g = G[idx];
            if (idx / k == idx % k) dg += g * g;
            else off += g * g;
        }
        double two[kChunk] = {off, dg};
        block_sums(two, 2, red, scratch);
        if (!(scratch[0] > 1e-30 * scratch[1])) break;
        for (int r = 0; r < K - 1; ++r) {
            if (tid < np) {
                int p, q;
                if (tid == 0) {
                    p = r;
                    q = K - 1;
                } else {
                    p = (r + tid) % (K - 1);
                    q = (r - tid + K - 1) % (K - 1);
                }
                double c = 1.0, s = 0.0;
                if (p < k && q < k) {
                    const double apq = G[p * k + q];
                    if (fabs(apq) > 1e-300) {
                        const double tau = (G[q * k + q] - G[p * k + p]) / (2.0 * apq);
                        double t;
                        if (fabs(tau) > 1e150) t = 0.5 / tau;
                        else t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                } else {
                    p = q = 0;
                }
                pp[tid] = p;
                qq[tid] = q;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            // rows p, q of G <- J^T G
            for (int idx = tid; idx < np * k; idx += kBoThreads) {
                const int pr = idx / k, col = idx - pr * k;
                const double c = cs[pr], s = sn[pr];
                if (s == 0.0) continue;
                const int p = pp[pr], q = qq[pr];
                const double gp = G[p * k + col], gq = G[q * k + col];
                G[p * k + col] = c * gp - s * gq;
                G[q * k + col] = s * gp + c * gq;
            }
            __syncthreads();
            // columns p, q of G <- G J and of Y <- Y J
            for (int idx = tid; idx < np * k; idx += kBoThreads) {
                const int pr = idx / k, row = idx - pr * k;
                const double c = cs[pr], s = sn[pr];
                if (s == 0.0) continue;
                const int p = pp[pr], q = qq[pr];
                const double gp = G[row * k + p], gq = G[row * k + q];
                G[row * k + p] = c * gp - s * gq;
                G[row * k + q] = s * gp + c * gq;
                const double yp = Y[row * k + p], yq = Y[row * k + q];
                Y[row * k + p] = c * yp - s * yq;
                Y[row * k + q] = s * yp + c * yq;
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        for (int a = 0; a < k; ++a) theta[a] = G[a * k + a];
        // ascending order (selection sort, columns of Y follow)
        for (int a = 0; a < k; ++a) {
            int best = a;
            for (int b = a + 1; b < k; ++b)
                if (theta[b] < theta[best]) best = b;
            if (best != a) {
                const double t = theta[a];
                theta[a] = theta[best];
                theta[best] = t;
                for (int row = 0; row < k; ++row) {
                    const double y = Y[row * k + a];
                    Y[row * k + a] = Y[row * k + best];
                    Y[row * k + best] = y;
                }
            }
        }
    }
    __syncthreads();
}

__device__ inline double unit_hash(unsigned long long x) {
    // splitmix64, then the top 53 bits as a double in [-1, 1)
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <int LOG2N>
__global__ void __launch_bounds__(kBoThreads) k_bo_lobpcg(BoArgs A) {
    constexpr int n = 1 << LOG2N;
    __shared__ double2 fb[n];
    __shared__ double red[kBoWaves * kChunk];
    __shared__ double dots[kBoMaxZ + 8];
    __shared__ double G[kBoMaxZ * kBoMaxZ];
    __shared__ double Y[kBoMaxZ * kBoMaxZ];
    __shared__ double theta[kBoMaxZ];
    __shared__ double scratch[kChunk];
    const int j = blockIdx.x, tid = threadIdx.x, m = A.m;
    double *V = A.ws + (size_t)j * A.ws_stride;
    double *Z = V + n;
    double *HZ = Z + (size_t)kBoMaxZ * n;
    double *X = HZ + (size_t)kBoMaxZ * n;
    double *P = X + (size_t)kBoMaxBlock * n;
    double *Wr = P + (size_t)kBoMaxBlock * n;
    const double Rj = A.Rv[j];

    // the clamped potential and its range on the grid
    double vmin = INFINITY, vmax = -INFINITY;
    bool finite = true;
    for (int e = tid; e < n; e += kBoThreads) {
        const double w = model_w(A.mp, A.r_min + e * A.h, Rj);
        V[e] = w;
        finite = finite && isfinite(w);
        vmin = fmin(vmin, w);
        vmax = fmax(vmax, w);
    }
    {
        double mm[kChunk] = {0};
        // range via sums of per-wave extrema: reduce max and -min with shuffles
        double a = vmax, b = -vmin;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a = fmax(a, __shfl_xor(a, off));
            b = fmax(b, __shfl_xor(b, off));
        }
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) {
            red[wave * kChunk] = a;
            red[wave * kChunk + 1] = b;
            red[wave * kChunk + 2] = finite ? 0.0 : 1.0;
        }
        __syncthreads();
        if (tid == 0) {
            double mx = red[0], mn = red[1], bad = red[2];
            for (int w = 1; w < kBoWaves; ++w) {
                mx = fmax(mx, red[w * kChunk]);
                mn = fmax(mn, red[w * kChunk + 1]);
                bad += red[w * kChunk + 2];
            }
            scratch[0] = mx + mn;    // max W - min W
            scratch[1] = bad;
        }
        __syncthreads();
        (void)mm;
    }
    const double cshift = fmax(1.0, scratch[0]);
    if (scratch[1] != 0.0) {
        if (tid == 0) atomicOr(&A.flags[kFlagNonfinite], 1);
        return;
    }
    __syncthreads();

    // starting block: pseudo-random columns, smoothed by the preconditioner
    for (int c = 0; c < m; ++c)
        for (int e = tid; e < n; e += kBoThreads)
            Wr[(size_t)c * n + e] = unit_hash(((unsigned long long)j << 40) ^ ((unsigned long long)c << 20) ^ e);
    __syncthreads();
    for (int c = 0; c < m; c += 2) {
        double *u = Wr + (size_t)c * n, *v = c + 1 < m ? u + n : nullptr;
        spectral_pair<LOG2N>(A, u, v, u, v, V, false, cshift, fb);
    }
    int kz = 0;
    for (int c = 0; c < m; ++c) kz = append_orthonormal<LOG2N>(Z, kz, Wr + (size_t)c * n, red, dots);

    int it = 0;
    double worst = INFINITY;
    for (;; ++it) {
        // h_e on the whole basis, afresh
        for (int c = 0; c < kz; c += 2) {
            const double *u = Z + (size_t)c * n, *v = c + 1 < kz ? u + n : nullptr;
            spectral_pair<LOG2N>(A, u, v, HZ + (size_t)c * n, v ? HZ + (size_t)(c + 1) * n : nullptr, V, true,
                                 cshift, fb);
        }
        // projected matrix G[a][b] = z_a . (h_e z_b), upper part, mirrored
        for (int a = 0; a < kz; ++a) {
            for (int b0 = a; b0 < kz; b0 += kChunk) {
                const int cc = min(kChunk, kz - b0);
                double part[kChunk] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int e = tid; e < n; e += kBoThreads) {
                    const double za = Z[(size_t)a * n + e];
#pragma unroll
                    for (int q = 0; q < kChunk; ++q)
                        if (q < cc) part[q] += za * HZ[(size_t)(b0 + q) * n + e];
                }
                block_sums(part, cc, red, dots);
                if (tid < cc) {
                    G[a * kz + b0 + tid] = dots[tid];
                    G[(b0 + tid) * kz + a] = dots[tid];
                }
                __syncthreads();
            }
        }
        jacobi(G, Y, kz, theta, red, scratch);
        const int mk = min(m, kz);
        // Ritz block, its residuals and the new directions
        for (int e = tid; e < n; e += kBoThreads) {
            for (int i = 0; i < mk; ++i) {
                double x = 0.0, hx = 0.0, p = 0.0;
                for (int a = 0; a < kz; ++a) {
                    const double y = Y[a * kz + i];
                    const double za = Z[(size_t)a * n + e];
                    x += za * y;
                    hx += HZ[(size_t)a * n + e] * y;
                    if (a >= m) p += za * y;
                }
                X[(size_t)i * n + e] = x;
                Wr[(size_t)i * n + e] = hx - theta[i] * x;
                P[(size_t)i * n + e] = p;
            }
        }
        __syncthreads();
        worst = 0.0;
        {
            double part[kChunk] = {0, 0, 0, 0, 0, 0, 0, 0};
            const int cw = min(A.nwant, mk);
            for (int e = tid; e < n; e += kBoThreads) {
#pragma unroll
                for (int q = 0; q < kChunk; ++q)
                    if (q < cw) {
                        const double r = Wr[(size_t)q * n + e];
                        part[q] += r * r;
                    }
            }
            block_sums(part, cw, red, dots);
            for (int q = 0; q < cw; ++q) worst = fmax(worst, sqrt(dots[q]));
            __syncthreads();
        }
        if (!(worst > A.tol) || it + 1 >= A.max_iter || !isfinite(worst)) break;
        // preconditioned residuals
        for (int c = 0; c < mk; c += 2) {
            double *u = Wr + (size_t)c * n, *v = c + 1 < mk ? u + n : nullptr;
            spectral_pair<LOG2N>(A, u, v, u, v, V, false, cshift, fb);
        }
        // new basis: the Ritz block, the preconditioned residuals, the directions
        kz = 0;
        for (int c = 0; c < mk; ++c) kz = append_orthonormal<LOG2N>(Z, kz, X + (size_t)c * n, red, dots);
        for (int c = 0; c < mk; ++c) kz = append_orthonormal<LOG2N>(Z, kz, Wr + (size_t)c * n, red, dots);
        if (it > 0)
            for (int c = 0; c < mk; ++c) kz = append_orthonormal<LOG2N>(Z, kz, P + (size_t)c * n, red, dots);
    }

    // output: grid normalisation, largest-magnitude entry positive
    const double scale = 1.0 / sqrt(A.h);
    for (int i = 0; i < A.nwant; ++i) {
        const double *x = X + (size_t)i * n;
        double best = -1.0;
        int bidx = n;
        for (int e = tid; e < n; e += kBoThreads) {
            const double ax = fabs(x[e]);
            if (ax > best) {
                best = ax;
                bidx = e;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bidx, off);
            if (ob > best || (ob == best && oi < bidx)) {
                best = ob;
                bidx = oi;
            }
        }
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) {
            red[wave * 2] = best;
            red[wave * 2 + 1] = (double)bidx;
        }
        __syncthreads();
        if (tid == 0) {
            double bb = red[0];
            int bi = (int)red[1];
            for (int w = 1; w < kBoWaves; ++w) {
                const double ob = red[2 * w];
                const int oi = (int)red[2 * w + 1];
                if (ob > bb || (ob == bb && oi < bi)) {
                    bb = ob;
                    bi = oi;
                }
            }
            scratch[0] = x[bi] < 0.0 ? -scale : scale;
        }
        __syncthreads();
        const double sg = scratch[0];
        double *dst = A.states + ((size_t)j * A.nwant + i) * n;
        for (int e = tid; e < n; e += kBoThreads) dst[e] = sg * x[e];
        if (tid == 0) A.energies[(size_t)j * A.nwant + i] = theta[i];
        __syncthreads();
    }
    if (tid == 0) {
        A.iters[j] = it + 1;
        A.resid[j] = worst;
    }
}

template <int LOG2N>
void launch_bo_t(const BoArgs &a, int nv, hipStream_t s) {
    hipLaunchKernelGGL(k_bo_lobpcg<LOG2N>, dim3(nv), dim3(kBoThreads), 0, s, a);
}

}  // namespace

}  // namespace icwf

// ---- C ABI (include/icwf_bo.h) -------------------------------------------------------------------

namespace {

bool bo_args_ok(const icwf_config *c, int32_t nv, int32_t ns, const char **why) {
    auto pow2 = [](int n) { return n > 0 && (n & (n - 1)) == 0; };
    if (!c) {
        *why = "config is NULL";
        return false;
    }
    if (!pow2(c->n_r) || c->n_r < 32 || c->n_r > 4096) {
        *why = "n_r must be a power of two in [32, 4096]";
        return false;
    }
    if (!(c->r_max > c->r_min) || !std::isfinite(c->r_min) || !std::isfinite(c->r_max) || !(c->m_r > 0) ||
        !std::isfinite(c->m_r)) {
        *why = "bad r box or m_r";
        return false;
    }
    if (c->model != ICWF_MODEL_SHIN_METIU && c->model != ICWF_MODEL_CAVITY) {
        *why = "unknown model";
        return false;
    }
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(c->model_params[i])) {
            *why = "model parameters must be finite";
            return false;
        }
    if (c->model == ICWF_MODEL_SHIN_METIU &&
        (!(c->model_params[1] > 0) || !(c->model_params[2] > 0) || !(c->model_params[3] > 0))) {
        *why = "Shin-Metiu softening lengths must be > 0";
        return false;
    }
    if (nv < 1 || nv > (1 << 20)) {
        *why = "n_values must be in [1, 2^20]";
        return false;
    }
    if (ns < 1 || ns > ICWF_BO_MAX_STATES || ns > c->n_r / 4) {
        *why = "n_states must be in [1, ICWF_BO_MAX_STATES] and at most n_r / 4";
        return false;
    }
    return true;
}

int block_size(int ns) { return ns + std::max(2, (ns + 1) / 2); }

// device layout: per-value slices, then the tables and the outputs
struct BoLayout {
    size_t slices, kin, tw, rvals, states, energies, iters, resid, flags, total;
};

BoLayout bo_layout(int n, int nv, int ns) {
    BoLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t at = off;
        off += bytes;
        return at;
    };
    L.slices = take(sizeof(double) * icwf::bo_stride(n) * nv);
    L.kin = take(sizeof(double) * n);
    L.tw = take(sizeof(double2) * (n / 2));
    L.rvals = take(sizeof(double) * nv);
    L.states = take(sizeof(double) * (size_t)nv * ns * n);
    L.energies = take(sizeof(double) * (size_t)nv * ns);
    L.iters = take(sizeof(int32_t) * nv);
    L.resid = take(sizeof(double) * nv);
    L.flags = take(sizeof(int32_t) * icwf::kNumFlags);
    L.total = (off + 255) & ~size_t(255);
    return L;
}

}  // namespace

extern "C" {

size_t icwf_bo_workspace_bytes(const icwf_config *cfg, int32_t n_values, int32_t n_states) {
    const char *why = nullptr;
    if (!bo_args_ok(cfg, n_values, n_states, &why)) return 0;
    return bo_layout(cfg->n_r, n_values, n_states).total;
}

icwf_status icwf_bo_states(const icwf_config *cfg, const double *R_values, int32_t n_values, int32_t n_states,
                           double *states, double *energies, void *workspace, size_t ws_bytes, void *hip_stream,
                           icwf_bo_info *info) {
    const char *why = nullptr;
    if (!bo_args_ok(cfg, n_values, n_states, &why)) return icwf::set_create_error(ICWF_EINVAL, why);
    if (!R_values) return icwf::set_create_error(ICWF_EINVAL, "R_values is NULL");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return icwf::set_create_error(ICWF_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    for (int j = 0; j < n_values; ++j)
        if (!std::isfinite(R_values[j])) return icwf::set_create_error(ICWF_ENONFINITE, "non-finite R value");
    const int n = cfg->n_r, nv = n_values, ns = n_states;
    const BoLayout L = bo_layout(n, nv, ns);
    if (ws_bytes < L.total) return icwf::set_create_error(ICWF_ENOMEM, "workspace smaller than icwf_bo_workspace_bytes()");
    const double h = (cfg->r_max - cfg->r_min) / n;
    double hbound = 0.0;
    std::vector<double> kin(n);
    std::vector<double2> tw(n / 2);
    for (int k = 0; k < n; ++k) {
        const int kk = (k <= n / 2) ? k : k - n;
        const double kw = 2.0 * M_PI * kk / (n * h);
        kin[k] = kw * kw / (2.0 * cfg->m_r);
        hbound = std::max(hbound, kin[k]);
    }
    for (int k = 0; k < n / 2; ++k) tw[k] = make_double2(std::cos(-2.0 * M_PI * k / n), std::sin(-2.0 * M_PI * k / n));
    char *base = reinterpret_cast<char *>(workspace);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    icwf::BoArgs a{};
    a.n = n;
    a.m = block_size(ns);
    a.nwant = ns;
    a.max_iter = (info && info->max_iter > 0) ? info->max_iter : 2000;
    // the bar: a few roundings of the largest kinetic term (the potential's
    // range is added where it is known to be larger, in the kernel's shift)
    a.tol = (info && info->tol > 0) ? info->tol : 32.0 * 2.220446049250313e-16 * std::max(1.0, hbound);
    a.r_min = cfg->r_min;
    a.h = h;
    a.mp.kind = cfg->model;
    for (int i = 0; i < 8; ++i) a.mp.p[i] = cfg->model_params[i];
    a.ws = reinterpret_cast<double *>(base + L.slices);
    a.ws_stride = icwf::bo_stride(n);
    a.kin = reinterpret_cast<const double *>(base + L.kin);
    a.tw = reinterpret_cast<const double2 *>(base + L.tw);
    a.states = reinterpret_cast<double *>(base + L.states);
    a.energies = reinterpret_cast<double *>(base + L.energies);
    a.iters = reinterpret_cast<int32_t *>(base + L.iters);
    a.resid = reinterpret_cast<double *>(base + L.resid);
    a.flags = reinterpret_cast<int32_t *>(base + L.flags);
    a.Rv = reinterpret_cast<const double *>(base + L.rvals);
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e == hipSuccess) return true;
        icwf::set_create_error(ICWF_EDEVICE, (std::string(what) + ": " + hipGetErrorString(e)).c_str());
        return false;
    };
    if (!hip_ok(hipMemcpyAsync(base + L.rvals, R_values, sizeof(double) * nv, hipMemcpyHostToDevice, st), "copy R") ||
        !hip_ok(hipMemcpyAsync(base + L.kin, kin.data(), sizeof(double) * n, hipMemcpyHostToDevice, st), "copy kin") ||
        !hip_ok(hipMemcpyAsync(base + L.tw, tw.data(), sizeof(double2) * (n / 2), hipMemcpyHostToDevice, st), "copy tw") ||
        !hip_ok(hipMemsetAsync(base + L.flags, 0, sizeof(int32_t) * icwf::kNumFlags, st), "clear flags"))
        return ICWF_EDEVICE;
    switch (n) {
        case 32: icwf::launch_bo_t<5>(a, nv, st); break;
        case 64: icwf::launch_bo_t<6>(a, nv, st); break;
        case 128: icwf::launch_bo_t<7>(a, nv, st); break;
        case 256: icwf::launch_bo_t<8>(a, nv, st); break;
        case 512: icwf::launch_bo_t<9>(a, nv, st); break;
        case 1024: icwf::launch_bo_t<10>(a, nv, st); break;
        case 2048: icwf::launch_bo_t<11>(a, nv, st); break;
        default: icwf::launch_bo_t<12>(a, nv, st); break;
    }
    if (!hip_ok(hipGetLastError(), "launch")) return ICWF_EDEVICE;
    std::vector<int32_t> iters(nv), flags(icwf::kNumFlags);
    std::vector<double> resid(nv);
    if ((states && !hip_ok(hipMemcpyAsync(states, base + L.states, sizeof(double) * (size_t)nv * ns * n,
                                          hipMemcpyDeviceToHost, st), "copy states")) ||
        (energies && !hip_ok(hipMemcpyAsync(energies, base + L.energies, sizeof(double) * (size_t)nv * ns,
                                            hipMemcpyDeviceToHost, st), "copy energies")) ||
        !hip_ok(hipMemcpyAsync(iters.data(), base + L.iters, sizeof(int32_t) * nv, hipMemcpyDeviceToHost, st), "copy iters") ||
        !hip_ok(hipMemcpyAsync(resid.data(), base + L.resid, sizeof(double) * nv, hipMemcpyDeviceToHost, st), "copy resid") ||
        !hip_ok(hipMemcpyAsync(flags.data(), base + L.flags, sizeof(int32_t) * icwf::kNumFlags, hipMemcpyDeviceToHost, st),
                "copy flags") ||
        !hip_ok(hipStreamSynchronize(st), "synchronise"))
        return ICWF_EDEVICE;
    if (flags[icwf::kFlagNonfinite]) return icwf::set_create_error(ICWF_ENONFINITE, "the model is singular on the grid");
    int worst_it = 0, unconv = 0;
    double worst_res = 0.0;
    for (int j = 0; j < nv; ++j) {
        worst_it = std::max(worst_it, iters[j]);
        worst_res = std::max(worst_res, resid[j]);
        if (!(resid[j] <= a.tol)) ++unconv;
    }
    if (info) {
        info->iterations = worst_it;
        info->max_residual = worst_res;
        info->unconverged = unconv;
    }
    if (unconv) return icwf::set_create_error(ICWF_ESOLVE, "some R values did not reach the residual bar");
    return ICWF_OK;
}

}  // extern "C"
