// The single-species matrices of Eq. 9 (9a, and the conditioned factors of
// 9c-9d) and the two-body contraction of Eq. 9b.
//
// Single species (k_zgemm): out[b][a] = h sum_k conj(X[b][k]) Y[a][k] for the
// pairs (X, Y) = (psi1, psi1) -> S1, (psi1, G1) -> E1, (psi2, psi2) -> S2,
// (psi2, G2) -> E2, where G is the ket weighted by the coupling potential at
// the ket's own trajectory: G1^a_i = W_c(r_i, R^a) psi1^a_i, G2^a_j =
// W_c(r^a, R_j) psi2^a_j.  Complex = four real FP64 MFMA products.
//
// Two-body (k_wc): Wc[b][a] = hr hR sum_j conj(psi2^b_j) psi2^a_j
//                             sum_i conj(psi1^b_i) psi1^a_i W_c(r_i, R_j)
// for b <= a (the matrix is Hermitian).  The inner i-sum is a real GEMM whose
// A operand, the pair product P1 = conj(psi1^b) psi1^a, is generated in
// registers (never stored) and whose B operand is the W_c table; the j-sum
// with the pair product P2 is fused into the epilogue of every 32-wide j
// tile.  FP64: v_mfma_f64_16x16x4 throughout.  Mixed: P1 and the table in
// FP32 on v_mfma_f32_16x16x4 with FP32 accumulation over i inside a j tile,
// the epilogue and the sum over j tiles in FP64.
#include <algorithm>

#include "icwf_plan.hpp"

namespace icwf {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- conditioned kets
__global__ void k_cond_kets(const double2 *__restrict__ psi, int n, double x_min, double h,
                            const double *__restrict__ cond_a, const double *__restrict__ cond_b, int species,
                            ModelParams mp, double2 *__restrict__ Ga, double2 *__restrict__ Gb, int Np,
                            const int32_t *__restrict__ flags, const long long *__restrict__ zoff, const ModelParams *__restrict__ mpd) {
    const long long zo_ = batch_offset(zoff);
    psi = zshift(psi, zo_);
    cond_a = zshift(cond_a, zo_);
    cond_b = zshift(cond_b, zo_);
    Ga = zshift(Ga, zo_);
    Gb = zshift(Gb, zo_);
    flags = zshift(flags, zo_);
    if (zoff) mp = *zshift(mpd, zo_);

    if (flags[kFlagHalt]) return;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)Np * n) return;
    const int a = (int)(idx / n);
    const int i = (int)(idx - (size_t)a * n);
    const double x = x_min + i * h;
    const double2 p = psi[idx];
    double wa, wb;
    if (species == 1) {
        wa = model_wc(mp, x, cond_a[a]);
        wb = model_wc(mp, x, cond_b[a]);
    } else {
        wa = model_wc(mp, cond_a[a], x);
        wb = model_wc(mp, cond_b[a], x);
    }
    Ga[idx] = cscale(p, wa);
    if (Gb) Gb[idx] = cscale(p, wb);
}

// ---------------------------------------------------------------- batched conj-NT complex GEMM
struct ZBatch {
    const double2 *X[6];
    const double2 *Y[6];
    double2 *out[6];
    int K[6];
    double scale[6];
};

// Work-group of 4 waves per 64 x 64 output tile, wave w on the 32 x 32
// quarter (rows 32 (w / 2), columns 32 (w % 2)) as 2 x 2 MFMA fragments with
// rows = b, columns = a, k the reduction index; lane l supplies
// A = X[b][k] and B = Y[a][k] with b, a = l % 16 of the fragment and
// k = l / 16 of the k step.  The 64 rows of X and of Y of a 16-wide k chunk are
// staged in LDS (two buffers: the coalesced global loads of chunk c + 1 are in
// flight while the matrix cores work on chunk c).  Hermitian outputs compute
// the upper tiles and write the lower ones as their conjugates.
constexpr int kZT = 64, kZKC = 16, kZLD = kZKC + 1;

// Entry z (wave-uniform) of a kernel-argument array, by selects: an indexed
// access would copy the whole argument struct to scratch.
template <typename T>
__device__ inline T zpick(const T (&a)[6], int z) {
    T r = a[0];
    r = z == 1 ? a[1] : r;
    r = z == 2 ? a[2] : r;
    r = z == 3 ? a[3] : r;
    r = z == 4 ? a[4] : r;
    r = z == 5 ? a[5] : r;
    return r;
}

template <bool BATCHED>
__global__ void __launch_bounds__(256, 2) k_zgemm(ZBatch zb, int Np, const int32_t *__restrict__ flags, int zcnt,
                                                  const long long *__restrict__ zoff) {
    // grid z: zcnt products of each simulation of the launch
    const int sim = BATCHED ? blockIdx.z / zcnt : 0, z = blockIdx.z - sim * zcnt;
    const long long zo_ = BATCHED ? batch_offset(zoff, sim) : 0;
    flags = zshift(flags, zo_);
    if (flags[kFlagHalt]) return;
    const int bt = blockIdx.y, at = blockIdx.x;
    const double2 *__restrict__ X = zshift(zpick(zb.X, z), zo_);
    const double2 *__restrict__ Y = zshift(zpick(zb.Y, z), zo_);
    const bool herm = X == Y;   // the output is Hermitian: upper tiles only
    if (herm && bt > at) return;
    __shared__ double2 sX[2][kZT][kZLD];
    __shared__ double2 sY[2][kZT][kZLD];
    const int K = zpick(zb.K, z);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int row = lane & 15, quarter = lane >> 4;
    const int b0 = bt * kZT, a0 = at * kZT;
    const int wb = 32 * (wave >> 1), wa = 32 * (wave & 1);
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            re[f][g] = dbl4{0, 0, 0, 0};
            im[f][g] = dbl4{0, 0, 0, 0};
        }
    // staging: element e = t + 256 m of a chunk is row e / 16, k e % 16
    const int srow = t >> 4, sk = t & 15;
    const double2 *xs = X + (size_t)(b0 + srow) * K + sk;   // rows srow + 16 m
    const double2 *ys = Y + (size_t)(a0 + srow) * K + sk;
    const size_t rstep = (size_t)16 * K;
    double2 rx0 = xs[0], rx1 = xs[rstep], rx2 = xs[2 * rstep], rx3 = xs[3 * rstep];
    double2 ry0 = ys[0], ry1 = ys[rstep], ry2 = ys[2 * rstep], ry3 = ys[3 * rstep];
    sX[0][srow][sk] = rx0;
    sX[0][srow + 16][sk] = rx1;
    sX[0][srow + 32][sk] = rx2;
    sX[0][srow + 48][sk] = rx3;
    sY[0][srow][sk] = ry0;
    sY[0][srow + 16][sk] = ry1;
    sY[0][srow + 32][sk] = ry2;
    sY[0][srow + 48][sk] = ry3;
    __syncthreads();
    const int nch = K / kZKC;
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nch;
        if (more) {
            const int k0 = (ch + 1) * kZKC;
            rx0 = xs[k0];
            rx1 = xs[rstep + k0];
            rx2 = xs[2 * rstep + k0];
            rx3 = xs[3 * rstep + k0];
            ry0 = ys[k0];
            ry1 = ys[rstep + k0];
            ry2 = ys[2 * rstep + k0];
            ry3 = ys[3 * rstep + k0];
        }
#pragma unroll
        for (int s4 = 0; s4 < kZKC / 4; ++s4) {
            const int kk = 4 * s4 + quarter;
            double2 xv[2], yv[2];
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                xv[f] = sX[buf][wb + 16 * f + row][kk];
                yv[f] = sY[buf][wa + 16 * f + row][kk];
            }
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    // conj(x) y = (xr yr + xi yi) + i (xr yi - xi yr)
                    re[f][g] = mfma(xv[f].x, yv[g].x, re[f][g]);
                    re[f][g] = mfma(xv[f].y, yv[g].y, re[f][g]);
                    im[f][g] = mfma(xv[f].x, yv[g].y, im[f][g]);
                    im[f][g] = mfma(-xv[f].y, yv[g].x, im[f][g]);
                }
        }
        if (more) {
            const int nb = buf ^ 1;
            sX[nb][srow][sk] = rx0;
            sX[nb][srow + 16][sk] = rx1;
            sX[nb][srow + 32][sk] = rx2;
            sX[nb][srow + 48][sk] = rx3;
            sY[nb][srow][sk] = ry0;
            sY[nb][srow + 16][sk] = ry1;
            sY[nb][srow + 32][sk] = ry2;
            sY[nb][srow + 48][sk] = ry3;
        }
        __syncthreads();
    }
    const double sc = zpick(zb.scale, z);
    double2 *out = zshift(zpick(zb.out, z), zo_);
    const bool mirror = herm && bt < at;
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = b0 + wb + 16 * f + mfma_row_f64(lane, v);
                const int a = a0 + wa + 16 * g + row;
                const double2 o = make_double2(sc * re[f][g][v], sc * im[f][g][v]);
                out[(size_t)b * Np + a] = o;
                if (mirror) out[(size_t)a * Np + b] = cconj(o);
            }
}

// ---------------------------------------------------------------- two-body contraction
template <typename T>
struct WcTraits;
template <>
struct WcTraits<double> {
    typedef dbl4 acc4;
    typedef double2 cplx;   // psi1 operand
};
template <>
struct WcTraits<float> {
    typedef flt4 acc4;
    typedef float2 cplx;    // FP32 copy of psi1 (written by the propagation)
};

__device__ inline void triangle_tile(int t, int *tb, int *ta) {
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    while (a * (a + 1) / 2 > t) --a;
    *ta = a;
    *tb = t - a * (a + 1) / 2;
}

// Block = 4 waves on a 16 (b) x 16 (a) tile of the upper triangle (tile
// index tb <= ta); wave w owns b = b_tile + 4w .. 4w + 3 against all 16 a.
// MFMA rows are a, columns are j, k is i; lane l supplies A = P1(b, a0 + l%16,
// i) and B = W_c(i, j0 + l%16) with i in the quarter l/16 of the current i
// chunk.  Each (j tile, i chunk) step stages the 32 psi1 rows of the tile and
// the W_c chunk in LDS (two buffers): the loads of step s + 1 are in flight
// while the matrix cores work on step s.  The j-sums of the epilogue go to
// LDS once per j tile.
//
// The staging goes straight from global memory into LDS (16 bytes per lane
// and load; no staging registers, four times fewer load instructions than
// 4-byte loads).  A load fills 64 consecutive 16-byte slots of a padded
// buffer: psi1 rows of 32 slots plus a pad slot (528 bytes), W_c rows of
// 16 slots plus one (FP64) or plus four (FP32), so that the operand reads
// stay free of bank conflicts; a lane whose slot is padding, or past the tile,
// loads an in-bounds entry that is never read.  FP32 takes the i of a chunk
// interleaved over the four lane quarters (i = 4 s + quarter at quad s), FP64
// in four consecutive runs (i = QS quarter + s).  FP32 accumulators take half
// the registers of FP64 ones, so its j tiles are 64 wide (each pair product
// feeds eight matrix products instead of four).
template <typename T>
struct WcChunk {
    static constexpr int KC = sizeof(T) == 8 ? 32 : 64;   // i per chunk (LDS budget: 2 blocks / CU)
    static constexpr int JT = sizeof(T) == 8 ? 32 : 64;   // j per tile
    static constexpr int JF = JT / 16;                    // 16-wide j fragments
    static constexpr int CPLX = 2 * sizeof(T);            // bytes of a psi1 entry
    static constexpr int LDA = 528 / CPLX;                 // padded psi1 row (entries): 33 slots
    static constexpr int LDW = sizeof(T) == 8 ? 34 : 80;   // padded W_c chunk row (entries)
    static constexpr bool INTERLEAVE = sizeof(T) == 4;
    static constexpr int ALOADS = (32 * 33 + 63) / 64;                 // loads per psi1 buffer
    static constexpr int AROWS = (64 * 16 * ALOADS + 527) / 528;       // rows the buffer holds
    static constexpr int WSLOTS = LDW * sizeof(T) / 16;                // slots per W_c row
    static constexpr int WDATA = JT * sizeof(T) / 16;                  // of which data
    static constexpr int WLOADS = (KC * WSLOTS + 63) / 64;
    static constexpr int WROWS = (64 * 16 * WLOADS + LDW * (int)sizeof(T) - 1) / (LDW * (int)sizeof(T));
};

typedef __attribute__((address_space(3))) void lds_void;

// Sum over the 16 lanes of a row of a double held by each lane (DPP
// rotations within the row); every lane of the row ends with the sum, lane
// 16 r in a fixed order.
template <int CTRL>
__device__ inline double dpp_rot(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double row16_sum(double x) {
    x += dpp_rot<0x128>(x);   // row_ror:8
    x += dpp_rot<0x124>(x);   // row_ror:4
    x += dpp_rot<0x122>(x);   // row_ror:2
    x += dpp_rot<0x121>(x);   // row_ror:1
    return x;
}

template <typename T, bool BATCHED>
__global__ void __launch_bounds__(256, 2) k_wc(const typename WcTraits<T>::cplx *__restrict__ psi1,
                                               const double2 *__restrict__ psi2,
                                               const T *__restrict__ wtab, int nr, int nR, double scale,
                                               double2 *__restrict__ Wc, int Np, int accumulate,
                                               int ntiles, int spq, int nparts, int32_t *__restrict__ queue,
                                               const int32_t *__restrict__ order, double2 *__restrict__ part,
                                               const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = BATCHED ? batch_offset(zoff) : 0;
    psi1 = zshift(psi1, zo_);
    psi2 = zshift(psi2, zo_);
    wtab = zshift(wtab, zo_);
    Wc = zshift(Wc, zo_);
    queue = zshift(queue, zo_);
    order = zshift(order, zo_);
    part = zshift(part, zo_);
    flags = zshift(flags, zo_);

    typedef typename WcTraits<T>::acc4 acc4;
    typedef typename WcTraits<T>::cplx C2;
    typedef WcChunk<T> CK;
    constexpr int KC = CK::KC, LDA = CK::LDA, LDW = CK::LDW, QS = KC / 4, JT = CK::JT, JF = CK::JF;
    constexpr int AROWS = CK::AROWS, WROWS = CK::WROWS;
    if (flags[kFlagHalt]) return;
    // two staging buffers as separate arrays: the compiler can then tell the
    // reads of one from the direct loads into the other
    __shared__ __align__(16) C2 sA0[AROWS][LDA], sA1[AROWS][LDA];   // rows 0..15: a rows, 16..31: b rows
    __shared__ __align__(16) T sW0[WROWS][LDW], sW1[WROWS][LDW];
    __shared__ double2 wl[4][4][16];   // [wave][b][a] block partial of Wc
    __shared__ int s_unit, s_queue, s_done;
    // persistent: the work-group takes upper-triangle tiles from queues until
    // none is left (fewer work-groups than CU slots leaves room for work on
    // another stream).  Queue q hands out the q-th eighth of the tile order
    // (blocks of neighbouring tiles); a work-group takes from the queue of
    // its own XCD first, then from the others.  The last spq tiles of each
    // queue come as nparts units each, one per nparts-th of the j tiles, so
    // that the final round ends with small pieces of work: each unit leaves
    // its partial sum in `part`, and the unit that completes last adds them
    // in part order (whatever the order of completion) and writes the tile.
    auto queue_range = [&](int q, int *lo, int *nfull, int *nsp) {
        *lo = (int)((long long)q * ntiles / kWcQueues);
        const int n = (int)((long long)(q + 1) * ntiles / kWcQueues) - *lo;
        *nsp = n < spq ? n : spq;
        *nfull = n - *nsp;
    };
    // the XCD this work-group runs on (its queue; any value is correct)
    const int xcd = __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kWcQueues - 1);   // HW_REG_XCC_ID
    for (;;) {
        if (threadIdx.x == 0) {
            int got = -1, gq = 0;
            for (int o = 0; o < kWcQueues && got < 0; ++o) {
                const int q = (xcd + o) & (kWcQueues - 1);
                int lo, nf, ns;
                queue_range(q, &lo, &nf, &ns);
                const int units = nf + ns * nparts;
                if (__hip_atomic_load(&queue[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= units) continue;
                const int k = atomicAdd(&queue[q], 1);
                if (k < units) {
                    got = k;
                    gq = q;
                }
            }
            s_unit = got;
            s_queue = gq;
        }
        __syncthreads();
        const int unit = s_unit, q = s_queue;
        __syncthreads();
        if (unit < 0) break;
        int lo, nfull, nsp;
        queue_range(q, &lo, &nfull, &nsp);
        int pos = lo + unit, half = -1, slot = 0;   // half: this unit's part of a split tile
        if (unit >= nfull) {
            const int j = unit - nfull;
            pos = lo + nfull + j / nparts;
            half = j - (j / nparts) * nparts;
            slot = q * spq + j / nparts;
        }
        int tb, ta;
        triangle_tile(order[pos], &tb, &ta);

        const int t = threadIdx.x;
        const int lane = t & 63, wave = t >> 6;
        const int row = lane & 15, quarter = lane >> 4;
        const int a_base = ta * 16;
        const int b_tile = tb * 16;
        const int b_base = b_tile + 4 * wave;

        for (int e = lane; e < 64; e += 64) wl[wave][e >> 4][e & 15] = make_double2(0, 0);

        const int nchunk = nr / KC, ntj = half < 0 ? nR / JT : nR / JT / nparts, nsteps = nchunk * ntj;
        const int jt0 = half > 0 ? half * ntj : 0;   // first j tile of this unit
        typedef C2 ATile[AROWS][LDA];
        typedef T WTile[WROWS][LDW];
        // tile row rr of the staging buffers: a rows first, then b rows
        auto tile_row = [&](int rr) { return rr < 16 ? a_base + rr : b_tile + rr - 16; };
        // one step's operands into (A, W): 64 slots per load, load m of
        // the buffer by wave m mod 4; slot -> (row, slot in the row)
        auto fetch = [&](int step, ATile &A, WTile &W) __attribute__((always_inline)) {
            const int jl = step / nchunk, ch = step - jl * nchunk, jt = jt0 + jl;
            const int i0 = ch * KC, j0 = jt * JT;
            const float4 *src_a = reinterpret_cast<const float4 *>(psi1);
            const float4 *src_w = reinterpret_cast<const float4 *>(wtab);
    #pragma unroll
            for (int m = 0; m < (CK::ALOADS + 3) / 4; ++m) {
                const int blk = 4 * m + wave;
                if (blk < CK::ALOADS) {
                    const int slot = 64 * blk + lane;
                    int rr = slot / 33, c = slot - 33 * rr;
                    if (rr >= 32) rr = 31;
                    if (c >= 32) c = 0;
                    // 16-byte units: a psi1 row is nr entries of CPLX bytes
                    const uint32_t off = (uint32_t)(((size_t)tile_row(rr) * nr + i0) * CK::CPLX / 16 + c);
                    __builtin_amdgcn_global_load_lds(reinterpret_cast<const float *>(src_a + off),
                                                     (lds_void *)(reinterpret_cast<char *>(&A[0][0]) + 1024 * blk), 16,
                                                     0, 0);
                }
            }
    #pragma unroll
            for (int m = 0; m < (CK::WLOADS + 3) / 4; ++m) {
                const int blk = 4 * m + wave;
                if (blk < CK::WLOADS) {
                    const int slot = 64 * blk + lane;
                    int ii = slot / CK::WSLOTS, c = slot - CK::WSLOTS * ii;
                    if (ii >= KC) ii = KC - 1;
                    if (c >= CK::WDATA) c = 0;
                    const uint32_t off = (uint32_t)(((size_t)(i0 + ii) * nR + j0) * sizeof(T) / 16 + c);
                    __builtin_amdgcn_global_load_lds(reinterpret_cast<const float *>(src_w + off),
                                                     (lds_void *)(reinterpret_cast<char *>(&W[0][0]) + 1024 * blk), 16,
                                                     0, 0);
                }
            }
        };
        // the loads have landed (vmcnt(0))
        auto stash = [&]() __attribute__((always_inline)) { __builtin_amdgcn_s_waitcnt(0x0f70); };

        acc4 acc[4][2][JF];   // [b][re/im][j fragment]
        // one (j tile, i chunk) step on the buffers (A, W); the next step's
        // operands are staged into (An, Wn) meanwhile
        auto body = [&](int step, ATile &A, WTile &W, ATile &An, WTile &Wn) __attribute__((always_inline)) {
            const int jl = step / nchunk, ch = step - jl * nchunk, jt = jt0 + jl;
            if (ch == 0) {
    #pragma unroll
                for (int bb = 0; bb < 4; ++bb)
    #pragma unroll
                    for (int c = 0; c < 2; ++c)
    #pragma unroll
                        for (int jf = 0; jf < JF; ++jf) acc[bb][c][jf] = acc4{0, 0, 0, 0};
            }
            if (step + 1 < nsteps) fetch(step + 1, An, Wn);
            // operands of i-quad s + 1 are read from LDS while the matrix
            // cores work on quad s
            C2 xa, xb[4];
            T w[JF];
            auto operands = [&](int s, C2 &oa, C2 (&ob)[4], T (&ow)[JF]) __attribute__((always_inline)) {
                const int col = CK::INTERLEAVE ? 4 * s + quarter : quarter * QS + s;
                oa = A[row][col];
    #pragma unroll
                for (int jf = 0; jf < JF; ++jf) ow[jf] = W[col][16 * jf + row];
    #pragma unroll
                for (int bb = 0; bb < 4; ++bb) ob[bb] = A[16 + 4 * wave + bb][col];
            };
            operands(0, xa, xb, w);
    #pragma unroll
            for (int s = 0; s < QS; ++s) {
                C2 na, nb[4];
                T nw[JF];
                if (s + 1 < QS) operands(s + 1, na, nb, nw);
    #pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    const C2 p = cmulc(xb[bb], xa);   // conj(psi1^b_i) psi1^a_i
                    const T pr = (T)p.x, pi = (T)p.y;
    #pragma unroll
                    for (int jf = 0; jf < JF; ++jf) {
                        acc[bb][0][jf] = mfma(pr, w[jf], acc[bb][0][jf]);
                        acc[bb][1][jf] = mfma(pi, w[jf], acc[bb][1][jf]);
                    }
                }
                if (s + 1 < QS) {
                    xa = na;
    #pragma unroll
                    for (int jf = 0; jf < JF; ++jf) w[jf] = nw[jf];
    #pragma unroll
                    for (int bb = 0; bb < 4; ++bb) xb[bb] = nb[bb];
                }
            }
            // keep the wait for the next step's operands after the matrix
            // products
            __builtin_amdgcn_sched_barrier(0);
            if (step + 1 < nsteps) stash();
            if (ch == nchunk - 1) {
                // epilogue: lane holds T(b, a = a_base + mfma_row(T, lane, v), j = j0 + 16 jf + row);
                // multiply by P2 = conj(psi2^b_j) psi2^a_j and sum over the 16 j of the fragment
                const int j0 = jt * JT;
                auto p2 = [&](int rr, int jj) { return psi2[(size_t)tile_row(rr) * nR + j0 + jj]; };
                // the a-row entries are loaded once for all b (two j
                // fragments), or again for each b (four: their registers are
                // needed for the accumulators)
                constexpr bool HOIST = JF <= 2;
                double2 p2a[HOIST ? JF : 1][4];
                if constexpr (HOIST) {
    #pragma unroll
                    for (int jf = 0; jf < JF; ++jf)
    #pragma unroll
                        for (int v = 0; v < 4; ++v) p2a[jf][v] = p2(mfma_row(T(0), lane, v), 16 * jf + row);
                }
                // one b at a time keeps the live registers low
    #pragma unroll
                for (int bb = 0; bb < 4; ++bb) {
                    double2 ws[4];
    #pragma unroll
                    for (int v = 0; v < 4; ++v) ws[v] = make_double2(0, 0);
    #pragma unroll
                    for (int jf = 0; jf < JF; ++jf) {
                        const double2 p2b = p2(16 + 4 * wave + bb, 16 * jf + row);
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const double2 pa = HOIST ? p2a[HOIST ? jf : 0][v] : p2(mfma_row(T(0), lane, v), 16 * jf + row);
                            const double2 P2 = cmulc(p2b, pa);
                            const double2 Tv = make_double2((double)acc[bb][0][jf][v], (double)acc[bb][1][jf][v]);
                            ws[v] = cadd(ws[v], cmul(P2, Tv));
                        }
                    }
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double2 x = make_double2(row16_sum(ws[v].x), row16_sum(ws[v].y));
                        if (row == 0) {
                            double2 &dst = wl[wave][bb][mfma_row(T(0), lane, v)];
                            dst = cadd(dst, x);
                        }
                    }
                }
            }
            __syncthreads();
        };
        fetch(0, sA0, sW0);
        stash();
        __syncthreads();
        // the buffers by name in each half of the loop (the reads of one need
        // not wait for the direct loads into the other)
        for (int step = 0; step < nsteps; step += 2) {
            body(step, sA0, sW0, sA1, sW1);
            if (step + 1 < nsteps) body(step + 1, sA1, sW1, sA0, sW0);
        }
        // write the 4 x 16 partials of this wave
        const int bb = lane >> 4, a = lane & 15;
        double2 *dst = Wc + (size_t)(b_base + bb) * Np + a_base + a;
        if (half < 0) {
            const double2 x = cscale(wl[wave][bb][a], scale);
            *dst = accumulate ? cadd(*dst, x) : x;
        } else {
            double2 *pp = part + (size_t)slot * nparts * 256 + wave * 64 + lane;
            pp[256 * half] = wl[wave][bb][a];
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0) s_done = atomicAdd(&queue[kWcQueues + slot], 1);
            __syncthreads();
            if (s_done == nparts - 1) {
                __threadfence();
                double2 acc = pp[0];
                for (int h = 1; h < nparts; ++h) acc = cadd(acc, pp[256 * h]);
                const double2 x = cscale(acc, scale);
                *dst = accumulate ? cadd(*dst, x) : x;
            }
        }
    }
}

// FP64 rank-K part of the two-body contraction:
//     Wc[b][a] (+)= hr hR sum_k alpha_k(b, a) beta_k(b, a),
//     alpha_k(b, a) = sum_i conj(psi1^b_i) psi1^a_i u_k(r_i),
//     beta_k(b, a)  = sum_j conj(psi2^b_j) psi2^a_j v_k(R_j),
// for W_c ~ sum_k u_k(r) v_k(R).  The pair tiles, queue, staging and pair
// products of k_wc, with the W_c table replaced by 16 rank factors at a time:
// MFMA rows = a, columns = the rank k of the chunk, reduction over i (then j
// with the psi2 rows); the epilogue multiplies the two products and sums over
// the chunk's ranks with 16-lane shuffles.  Ranks above K have zero factors.
constexpr int kSepKC = 32;   // grid points per staged chunk

// One factor product of a rank chunk: acc[bb][re/im] (rows a, columns k) =
// sum_i conj(X^b_i) X^a_i F[k0 + k][i] for the wave's four b rows.
__device__ inline void sep_pass(dbl4 (&acc)[4][2], const double2 *__restrict__ X, const double *__restrict__ F,
                                int n, int k0, int a_base, int b_tile, double2 (*sA)[32][kSepKC + 1],
                                double (*sF)[kSepKC][17]) {
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int row = lane & 15, quarter = lane >> 4;
    constexpr int QS = kSepKC / 4;
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
        acc[bb][0] = dbl4{0, 0, 0, 0};
        acc[bb][1] = dbl4{0, 0, 0, 0};
    }
    const int nchunk = n / kSepKC;
    // staging: element e = t + 256 m of the 32 psi rows x 32 points (m < 4) and
    // of the 32 points x 16 ranks of the factors (m < 2)
    double2 ra0, ra1, ra2, ra3;
    double rf0, rf1;
    const int rr0 = t >> 5, cc = t & 31;
    const int ii0 = t >> 4, kk = t & 15;
    const double2 *xrow[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int rr = rr0 + 8 * m;
        xrow[m] = X + (size_t)(rr < 16 ? a_base + rr : b_tile + rr - 16) * n + cc;
    }
    const double *frow = F + (size_t)(k0 + kk) * n + ii0;
    ra0 = xrow[0][0];
    ra1 = xrow[1][0];
    ra2 = xrow[2][0];
    ra3 = xrow[3][0];
    rf0 = frow[0];
    rf1 = frow[16];
    sA[0][rr0][cc] = ra0;
    sA[0][rr0 + 8][cc] = ra1;
    sA[0][rr0 + 16][cc] = ra2;
    sA[0][rr0 + 24][cc] = ra3;
    sF[0][ii0][kk] = rf0;
    sF[0][ii0 + 16][kk] = rf1;
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nchunk;
        if (more) {
            const int o = (ch + 1) * kSepKC;
            ra0 = xrow[0][o];
            ra1 = xrow[1][o];
            ra2 = xrow[2][o];
            ra3 = xrow[3][o];
            rf0 = frow[o];
            rf1 = frow[o + 16];
        }
#pragma unroll 2
        for (int s = 0; s < QS; ++s) {
            const int col = quarter * QS + s;
            const double2 xa = sA[buf][row][col];
            const double f = sF[buf][col][row];
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const double2 p = cmulc(sA[buf][16 + 4 * wave + bb][col], xa);   // conj(X^b_i) X^a_i
                acc[bb][0] = mfma(p.x, f, acc[bb][0]);
                acc[bb][1] = mfma(p.y, f, acc[bb][1]);
            }
        }
        if (more) {
            const int nb = buf ^ 1;
            sA[nb][rr0][cc] = ra0;
            sA[nb][rr0 + 8][cc] = ra1;
            sA[nb][rr0 + 16][cc] = ra2;
            sA[nb][rr0 + 24][cc] = ra3;
            sF[nb][ii0][kk] = rf0;
            sF[nb][ii0 + 16][kk] = rf1;
        }
        __syncthreads();
    }
}

template <bool BATCHED>
__global__ void __launch_bounds__(256, 2) k_wc_sep(const double2 *__restrict__ psi1, const double2 *__restrict__ psi2,
                                                   const double *__restrict__ U, const double *__restrict__ V,
                                                   int kpad, int nr, int nR, double scale,
                                                   double2 *__restrict__ Wc, int Np, int accumulate, int ntiles,
                                                   int32_t *__restrict__ queue, const int32_t *__restrict__ order,
                                                   const int32_t *__restrict__ flags, const long long *__restrict__ zoff) {
    const long long zo_ = BATCHED ? batch_offset(zoff) : 0;
    psi1 = zshift(psi1, zo_);
    psi2 = zshift(psi2, zo_);
    U = zshift(U, zo_);
    V = zshift(V, zo_);
    Wc = zshift(Wc, zo_);
    queue = zshift(queue, zo_);
    order = zshift(order, zo_);
    flags = zshift(flags, zo_);

    if (flags[kFlagHalt]) return;
    __shared__ double2 sA[2][32][kSepKC + 1];
    __shared__ double sF[2][kSepKC][17];
    __shared__ double2 wl[4][4][16];     // [wave][b][a] block partial of Wc
    __shared__ int s_tile;
    // tiles from the per-XCD queues over the blocked tile order, as k_wc
    const int xcd = __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kWcQueues - 1);   // HW_REG_XCC_ID
    for (;;) {
        if (threadIdx.x == 0) {
            int got = -1;
            for (int o = 0; o < kWcQueues && got < 0; ++o) {
                const int q = (xcd + o) & (kWcQueues - 1);
                const int lo = (int)((long long)q * ntiles / kWcQueues);
                const int n = (int)((long long)(q + 1) * ntiles / kWcQueues) - lo;
                if (__hip_atomic_load(&queue[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) continue;
                const int k = atomicAdd(&queue[q], 1);
                if (k < n) got = lo + k;
            }
            s_tile = got;
        }
        __syncthreads();
        const int pos = s_tile;
        __syncthreads();
        if (pos < 0) break;
        int tb, ta;
        triangle_tile(order[pos], &tb, &ta);
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
        const int row = lane & 15;
        const int a_base = ta * 16, b_tile = tb * 16, b_base = b_tile + 4 * wave;
        wl[wave][lane >> 4][lane & 15] = make_double2(0, 0);
        for (int k0 = 0; k0 < kpad; k0 += 16) {
            dbl4 acc1[4][2], acc2[4][2];
            sep_pass(acc1, psi1, U, nr, k0, a_base, b_tile, sA, sF);
            sep_pass(acc2, psi2, V, nR, k0, a_base, b_tile, sA, sF);
#pragma unroll
            for (int bb = 0; bb < 4; ++bb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // lane: a = a_base + mfma_row(lane, v), rank k0 + row
                    double2 x = cmul(make_double2(acc1[bb][0][v], acc1[bb][1][v]),
                                     make_double2(acc2[bb][0][v], acc2[bb][1][v]));
#pragma unroll
                    for (int off = 8; off > 0; off >>= 1) {
                        x.x += __shfl_xor(x.x, off, 16);
                        x.y += __shfl_xor(x.y, off, 16);
                    }
                    if (row == 0) {
                        double2 &dst = wl[wave][bb][mfma_row_f64(lane, v)];
                        dst = cadd(dst, x);
                    }
                }
        }
        {
            const int bb = lane >> 4, a = lane & 15;
            const double2 x = cscale(wl[wave][bb][a], scale);
            double2 *dst = Wc + (size_t)(b_base + bb) * Np + a_base + a;
            *dst = accumulate ? cadd(*dst, x) : x;
        }
    }
}

}  // namespace

std::vector<int32_t> wc_tile_order(int Np) {
    const int T = Np / 16, S = 8, nS = (T + S - 1) / S;
    std::vector<int32_t> ord;
    ord.reserve((size_t)T * (T + 1) / 2);
    for (int sb = 0; sb < nS; ++sb)
        for (int sa = sb; sa < nS; ++sa)
            for (int tb = sb * S; tb < std::min(T, sb * S + S); ++tb)
                for (int ta = std::max(tb, sa * S); ta < std::min(T, sa * S + S); ++ta)
                    ord.push_back(ta * (ta + 1) / 2 + tb);
    return ord;
}

void launch_cond_kets(const Dims &d, const Bufs &b, hipStream_t s, bool next) {
    const int Np = padded(d.N);
    size_t tot = (size_t)Np * d.nr;
    hipLaunchKernelGGL(k_cond_kets, dim3((unsigned)((tot + 255) / 256), 1, d.batch), dim3(256), 0, s, b.psi1, d.nr,
                       d.r_min, d.hr, b.R, b.R_new, 1, d.mp, b.G1a, next ? b.G1b : nullptr, Np, b.flags, d.zoff, d.mpd);
    tot = (size_t)Np * d.nR;
    hipLaunchKernelGGL(k_cond_kets, dim3((unsigned)((tot + 255) / 256), 1, d.batch), dim3(256), 0, s, b.psi2, d.nR,
                       d.R_min, d.hR, b.r, b.r_new, 2, d.mp, b.G2a, next ? b.G2b : nullptr, Np, b.flags, d.zoff, d.mpd);
}

void launch_cond_kets_next(const Dims &d, const Bufs &b, hipStream_t s) {
    const int Np = padded(d.N);
    size_t tot = (size_t)Np * d.nr;
    hipLaunchKernelGGL(k_cond_kets, dim3((unsigned)((tot + 255) / 256), 1, d.batch), dim3(256), 0, s, b.psi1, d.nr,
                       d.r_min, d.hr, b.R_new, b.R_new, 1, d.mp, b.G1b, nullptr, Np, b.flags, d.zoff, d.mpd);
    tot = (size_t)Np * d.nR;
    hipLaunchKernelGGL(k_cond_kets, dim3((unsigned)((tot + 255) / 256), 1, d.batch), dim3(256), 0, s, b.psi2, d.nR,
                       d.R_min, d.hR, b.r_new, b.r_new, 2, d.mp, b.G2b, nullptr, Np, b.flags, d.zoff, d.mpd);
}

void launch_single_species(const Dims &d, const Bufs &b, bool both, hipStream_t s, int parts) {
    const int Np = padded(d.N);
    ZBatch zb{};
    int c = 0;
    auto add = [&](const double2 *X, const double2 *Y, double2 *o, int K, double sc) {
        zb.X[c] = X;
        zb.Y[c] = Y;
        zb.out[c] = o;
        zb.K[c] = K;
        zb.scale[c] = sc;
        ++c;
    };
    if (parts & kSingleOverlaps) {
        add(b.psi1, b.psi1, b.S1, d.nr, d.hr);
        add(b.psi2, b.psi2, b.S2, d.nR, d.hR);
    }
    if (parts & kSingleCouplings) {
        add(b.psi1, b.G1a, b.E1a, d.nr, d.hr);
        add(b.psi2, b.G2a, b.E2a, d.nR, d.hR);
        if (both) {
            add(b.psi1, b.G1b, b.E1b, d.nr, d.hr);
            add(b.psi2, b.G2b, b.E2b, d.nR, d.hR);
        }
    }
    if (c == 0) return;
    hipLaunchKernelGGL(d.zoff ? k_zgemm<true> : k_zgemm<false>, dim3(Np / kZT, Np / kZT, c * d.batch), dim3(256), 0, s,
                       zb, Np, b.flags, c, d.zoff);
}

void launch_single_species_next(const Dims &d, const Bufs &b, hipStream_t s) {
    const int Np = padded(d.N);
    ZBatch zb{};
    zb.X[0] = b.psi1;
    zb.Y[0] = b.G1b;
    zb.out[0] = b.E1b;
    zb.K[0] = d.nr;
    zb.scale[0] = d.hr;
    zb.X[1] = b.psi2;
    zb.Y[1] = b.G2b;
    zb.out[1] = b.E2b;
    zb.K[1] = d.nR;
    zb.scale[1] = d.hR;
    hipLaunchKernelGGL(d.zoff ? k_zgemm<true> : k_zgemm<false>, dim3(Np / kZT, Np / kZT, 2 * d.batch), dim3(256), 0, s,
                       zb, Np, b.flags, 2, d.zoff);
}

void launch_wc(const Dims &d, const Bufs &b, hipStream_t s) {
    const int Np = padded(d.N);
    const int T16 = Np / 16;
    const int blocks = T16 * (T16 + 1) / 2;
    const double scale = d.hr * d.hR;
    // the last round of tiles split in kWcParts (fewer where R has fewer j
    // tiles)
    const int grid = std::min(blocks, d.wc_grid);
    auto split = [&](int jt, int *nparts, int *spq) {
        *nparts = std::min(kWcParts, d.nR / jt);
        const int nsplit = *nparts >= 2 ? std::min(grid, wc_split_tiles(Np)) : 0;
        *spq = wc_split_per_queue(nsplit);   // split tiles per queue
    };
    int nparts, spq;
    // the FP32 pass tiles the grid in chunks of 64 x 64 points: smaller grids
    // take the dense FP64 contraction of the whole table instead
    const bool fp32_fits = d.nr >= WcChunk<float>::KC && d.nR >= WcChunk<float>::JT;
    if (d.prec == 1 && fp32_fits) {
        // mixed: FP32 matrix cores on the residual of the rank-K split, FP64 rank-K part added
        // (the FP32 pass only where the residual is above the table's rounding)
        if (d.fp32_residual) {
            split(WcChunk<float>::JT, &nparts, &spq);
            launch_fill_i32(b.wc_queue, kWcQueues + kWcQueues * spq, 0, s, d.batch, d.zoff);
            hipLaunchKernelGGL((d.zoff ? k_wc<float, true> : k_wc<float, false>), dim3(grid, 1, d.batch), dim3(256), 0, s, b.psi1_f32, b.psi2, b.wc32, d.nr,
                               d.nR, scale, b.Wc, Np, 0, blocks, spq, nparts, b.wc_queue, b.wc_order, b.wc_part,
                               b.flags, d.zoff);
        }
        if (d.lr_rank > 0) {
            launch_fill_i32(b.wc_queue, kWcQueues, 0, s, d.batch, d.zoff);
            hipLaunchKernelGGL(d.zoff ? k_wc_sep<true> : k_wc_sep<false>, dim3(std::min(blocks, d.wc_grid), 1, d.batch), dim3(256), 0, s, b.psi1,
                               b.psi2, b.lr_u, b.lr_v, (d.lr_rank + 15) / 16 * 16, d.nr, d.nR, scale, b.Wc, Np,
                               d.fp32_residual ? 1 : 0, blocks, b.wc_queue, b.wc_order, b.flags, d.zoff);
        }
    } else if (d.prec == 2) {
        // separable: the whole contraction through the sum of products (assigns Wc)
        launch_fill_i32(b.wc_queue, kWcQueues, 0, s, d.batch, d.zoff);
        hipLaunchKernelGGL(d.zoff ? k_wc_sep<true> : k_wc_sep<false>, dim3(std::min(blocks, d.wc_grid), 1, d.batch), dim3(256), 0, s, b.psi1, b.psi2,
                           b.lr_u, b.lr_v, (d.lr_rank + 15) / 16 * 16, d.nr, d.nR, scale, b.Wc, Np, 0, blocks,
                           b.wc_queue, b.wc_order, b.flags, d.zoff);
    } else {
        split(WcChunk<double>::JT, &nparts, &spq);
        launch_fill_i32(b.wc_queue, kWcQueues + kWcQueues * spq, 0, s, d.batch, d.zoff);
        hipLaunchKernelGGL((d.zoff ? k_wc<double, true> : k_wc<double, false>), dim3(grid, 1, d.batch), dim3(256), 0, s, b.psi1, b.psi2, b.wc64, d.nr, d.nR,
                           scale, b.Wc, Np, 0, blocks, spq, nparts, b.wc_queue, b.wc_order, b.wc_part, b.flags,
                           d.zoff);
    }
}

}  // namespace icwf
