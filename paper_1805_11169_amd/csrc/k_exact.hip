// Propagation of the full two-dimensional wavefunction Psi(r_i, R_j) (Eq. 1
// with the Hamiltonian of Eq. 2 on the product grid), by the same Strang
// split operator the conditional wavefunctions use, in two dimensions:
//
//     Psi <- e^{-i W dt/2} IFFT2[ e^{-i (k_r^2/2m_r + k_R^2/2m_R) dt} FFT2[ e^{-i W dt/2} Psi ] ].
//
// This is the reference the ansatz of Eq. 7 converges to as N grows; it
// stores n_r n_R values where the method stores N (n_r + n_R).
//
// A call of n steps makes 2n + 1 passes over the state, each reading it once
// and writing it once.  Between passes the state stays transposed, in tmp
// [n_R][n_r], so that the r transforms read and write whole rows and only the
// R passes, several grid rows at a time, go through columns:
//   rows_fwd   rows i of Psi [n_r][n_R]: half-step potential phase, FFT along
//              R, written as columns i of tmp;
//   cols       rows k_R of tmp, in place: FFT along r, kinetic phase (a
//              product of one factor per coordinate; the nuclear one carries
//              the 1/(n_r n_R) of the inverse transform), inverse FFT along r;
//   rows_mid   columns i of tmp between two steps, in place: inverse FFT along
//              R, the half-step phase of the step that ends and of the step
//              that begins (two multiplications, as two half steps), FFT
//              along R;
//   rows_inv   after the last step: columns i of tmp, inverse FFT along R,
//              half-step phase, written as rows i of Psi.
// So n steps run rows_fwd, (cols, rows_mid) n - 1 times, cols, rows_inv.
//
// Each row of n = 2^L points is transformed by T = n/16 threads holding 16
// values each in registers, v[m] = element j + T m in thread j: a Stockham
// autosort FFT of ceil(L/4) passes, radix 16 but the last (radix n/16^(P-1)).
// A pass of radix R with Ns points per finished sub-transform combines R of
// them: butterfly b (< n/R) takes elements b + t n/R (t < R), multiplies
// element t by e^{-/+2 pi i t (b mod Ns) / (R Ns)}, takes the R-point DFT and
// sends output s to position (b - b mod Ns) R + b mod Ns + s Ns.  Thread j
// runs butterflies j + T u (u < 16/R), whose inputs are exactly its own 16
// values; the outputs go through LDS to the next pass (one exchange), except
// in the last pass, where output s of butterfly j + T u is element
// j + T (u + 16 s/R), again the thread's own: the transform ends in
// registers in the order it starts from, so the kinetic phase and the inverse
// transform follow without an exchange.  A 4096-point transform makes two
// exchanges (the previous design, radix 4 through LDS, made six).
//
// LDS holds one padded row per row of the work-group (n + n/16 values;
// element i at i + i/16, so that the radix-16 writes of consecutive threads,
// 16 values apart, fall in different banks): 69.6 KB for a 4096-point row or
// eight 512-point rows, two work-groups per CU.
//
// Work-groups are numbered XCD-major (work-group b runs on XCD b mod 8 and is
// given rows of block (b mod 8) G/8 + b/8), so that the grid rows whose
// column elements share a 128-byte line of tmp go through one L2.

#include <hip/hip_runtime.h>

#include "icwf_device.hpp"
#include "icwf_plan.hpp"

namespace icwf {
namespace {

// cos(2 pi e / 16), sin(2 pi e / 16) for e < 16, from cos(pi/8), sin(pi/8)
// and sqrt(1/2)
constexpr double kC8 = 0.92387953251128675613;   // cos(pi/8)
constexpr double kS8 = 0.38268343236508977173;   // sin(pi/8)
constexpr double kH2 = 0.70710678118654752440;   // sqrt(1/2)

__device__ __forceinline__ constexpr double cos16(int e) {
    constexpr double c[16] = {1.0, kC8, kH2, kS8, 0.0, -kS8, -kH2, -kC8, -1.0, -kC8, -kH2, -kS8, 0.0, kS8, kH2, kC8};
    return c[e & 15];
}
__device__ __forceinline__ constexpr double sin16(int e) {
    return cos16(e + 12);   // sin x = cos(x - pi/2)
}

// a e^{-/+ 2 pi i e / 16}; exact for e a multiple of 4
template <int E, bool INV>
__device__ __forceinline__ double2 rot16(double2 a) {
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return a;
    } else if constexpr (e == 8) {
        return make_double2(-a.x, -a.y);
    } else if constexpr (e == 4 || e == 12) {
        if constexpr ((e == 4) != INV) return make_double2(a.y, -a.x);   // times -i
        else return make_double2(-a.y, a.x);                            // times +i
    } else {
        constexpr double c = cos16(e), s = INV ? sin16(e) : -sin16(e);
        return make_double2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

template <int... I>
struct Seq {};
template <int N, int... I>
struct MakeSeq : MakeSeq<N - 1, N - 1, I...> {};
template <int... I>
struct MakeSeq<0, I...> {
    using type = Seq<I...>;
};
// f(std::integral_constant-like tag) for I = 0 .. N-1, unrolled at compile time
template <int V>
struct Int {
    static constexpr int value = V;
};
template <typename F, int... I>
__device__ __forceinline__ void for_each(F &&f, Seq<I...>) {
    (f(Int<I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void unroll(F &&f) {
    for_each(f, typename MakeSeq<N>::type{});
}

// In-register DFT of R = 2, 4, 8, 16 points: x[k] <- sum_m x[m] e^{-/+ 2 pi i m k / R}.
// R = R1 R2 (R2 = 4): m = R2 m1 + m2, k = k1 + R1 k2; R2 DFTs of R1 points over
// m1, the factors e^{-/+ 2 pi i m2 k1 / R}, R1 DFTs of R2 points over m2.
template <int R, bool INV>
__device__ __forceinline__ void dft(double2 (&x)[R]) {
    if constexpr (R == 2) {
        const double2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]), a2 = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        const double2 a3 = INV ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);   // -/+ i d
        x[0] = cadd(a0, a2);
        x[1] = cadd(a1, a3);
        x[2] = csub(a0, a2);
        x[3] = csub(a1, a3);
    } else {
        constexpr int R2 = 4, R1 = R / 4;
        double2 y[R];
        unroll<R2>([&](auto m2) {
            double2 t[R1];
            unroll<R1>([&](auto m1) { t[m1.value] = x[R2 * m1.value + m2.value]; });
            dft<R1, INV>(t);
            unroll<R1>([&](auto k1) {
                y[k1.value * R2 + m2.value] = rot16<(16 / R) * m2.value * k1.value, INV>(t[k1.value]);
            });
        });
        unroll<R1>([&](auto k1) {
            double2 t[R2];
            unroll<R2>([&](auto m2) { t[m2.value] = y[k1.value * R2 + m2.value]; });
            dft<R2, INV>(t);
            unroll<R2>([&](auto k2) { x[k1.value + R1 * k2.value] = t[k2.value]; });
        });
    }
}

__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Twiddles of the radix-16 passes after the first: e^{-2 pi i r k / (16 Ns)}
// for r < 16, k = j mod Ns.  The table entries for r = 1, 2, 4, 8 are loaded
// once per kernel (they serve the forward transform and, conjugated, the
// inverse one); the other eleven are their products (at most three
// roundings each).
template <int LOG2N>
struct TwBase {
    double2 w[2][4];   // passes 1 and 2 (Ns = 16, 256): r = 1, 2, 4, 8
};
template <int LOG2N>
__device__ __forceinline__ void load_tw_base(TwBase<LOG2N> &tb, const double2 *__restrict__ tw, int j) {
    constexpr int n = 1 << LOG2N, P = (LOG2N + 3) / 4, RL = 1 << (LOG2N - 4 * (P - 1));
    unroll<2>([&](auto p) {
        constexpr int NS = p.value == 0 ? 16 : 256;
        constexpr bool radix16 = p.value + 2 < P || (p.value + 2 == P && RL == 16);
        if constexpr (radix16) {
            const int base = (j & (NS - 1)) * (n / (16 * NS));
            unroll<4>([&](auto b) { tb.w[p.value][b.value] = tw[(1 << b.value) * base]; });
        }
    });
}
template <bool INV>
__device__ __forceinline__ void twiddles16(const double2 (&b)[4], double2 (&w)[16]) {
    const double2 w1 = INV ? cconj(b[0]) : b[0], w2 = INV ? cconj(b[1]) : b[1], w4 = INV ? cconj(b[2]) : b[2],
                  w8 = INV ? cconj(b[3]) : b[3];
    const double2 w3 = cmul(w1, w2), w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
    w[1] = w1;
    w[2] = w2;
    w[3] = w3;
    w[4] = w4;
    w[5] = w5;
    w[6] = w6;
    w[7] = w7;
    w[8] = w8;
    w[9] = cmul(w1, w8);
    w[10] = cmul(w2, w8);
    w[11] = cmul(w3, w8);
    w[12] = cmul(w4, w8);
    w[13] = cmul(w5, w8);
    w[14] = cmul(w6, w8);
    w[15] = cmul(w7, w8);
}

// One Stockham pass of radix RP (NS points per finished sub-transform) on a
// row of n = 2^LOG2N points held as v[m] = element j + T m of thread j.  Not
// LAST: the outputs go to the row's LDS (padded) and come back in the same
// distribution; LAST: they stay in v.  tw[m] = e^{-2 pi i m / n}; base: the
// pass's loaded twiddles when RP = 16 and NS > 1.
template <int LOG2N, int RP, int NS, bool INV, bool LAST>
__device__ __forceinline__ void fft_pass(double2 (&v)[16], double2 *row, const double2 *__restrict__ tw,
                                         const double2 (&base)[4], int j) {
    constexpr int n = 1 << LOG2N, T = n / 16, U = 16 / RP, STRIDE = n / (RP * NS);
    double2 w[U][RP];
    if constexpr (NS > 1 && RP == 16) {
        twiddles16<INV>(base, w[0]);
    } else if constexpr (NS > 1) {
        unroll<U>([&](auto u) {
            const int k = (j + T * u.value) & (NS - 1);
            unroll<RP - 1>([&](auto r) {
                double2 t = tw[(r.value + 1) * k * STRIDE];
                if (INV) t.y = -t.y;
                w[u.value][r.value + 1] = t;
            });
        });
    }
    unroll<U>([&](auto u) {
        double2 x[RP];
        unroll<RP>([&](auto r) {
            x[r.value] = v[u.value + r.value * U];
            if constexpr (NS > 1 && r.value > 0) x[r.value] = cmul(x[r.value], w[u.value][r.value]);
        });
        dft<RP, INV>(x);
        if constexpr (LAST) {
            unroll<RP>([&](auto s) { v[u.value + s.value * U] = x[s.value]; });
        } else {
            const int b = j + T * u.value, k = b & (NS - 1), o = (b - k) * RP + k;
            unroll<RP>([&](auto s) { row[pad16(o + s.value * NS)] = x[s.value]; });
        }
    });
    if constexpr (!LAST) {
        __syncthreads();
        unroll<16>([&](auto m) { v[m.value] = row[pad16(j + T * m.value)]; });
        __syncthreads();
    }
}

// The whole n-point transform, unscaled: ceil(LOG2N/4) passes, radix 16 but
// the last.  Ends with the result in v, in the order it started from.
// before_last() runs after the last exchange (a place to issue loads whose
// latency the last pass hides).
template <int LOG2N, bool INV, typename F>
__device__ __forceinline__ void fft_row(double2 (&v)[16], double2 *row, const double2 *__restrict__ tw,
                                        const TwBase<LOG2N> &tb, int j, F &&before_last) {
    static_assert(LOG2N >= 5 && LOG2N <= 12, "grid sizes 32 ... 4096");
    constexpr int P = (LOG2N + 3) / 4;
    constexpr int RL = 1 << (LOG2N - 4 * (P - 1));
    if constexpr (P == 2) {
        fft_pass<LOG2N, 16, 1, INV, false>(v, row, tw, tb.w[0], j);
        before_last();
        fft_pass<LOG2N, RL, 16, INV, true>(v, row, tw, tb.w[0], j);
    } else {
        fft_pass<LOG2N, 16, 1, INV, false>(v, row, tw, tb.w[0], j);
        fft_pass<LOG2N, 16, 16, INV, false>(v, row, tw, tb.w[0], j);
        before_last();
        fft_pass<LOG2N, RL, 256, INV, true>(v, row, tw, tb.w[1], j);
    }
}
template <int LOG2N, bool INV>
__device__ __forceinline__ void fft_row(double2 (&v)[16], double2 *row, const double2 *__restrict__ tw,
                                        const TwBase<LOG2N> &tb, int j) {
    fft_row<LOG2N, INV>(v, row, tw, tb, j, [] {});
}

// Rows per work-group: the wide variant (up to 69.6 KB of LDS, up to eight
// rows, so that a transposed write fills 128 bytes) and the narrow one (one
// wave, or one row), for grids with few rows.
template <int L>
constexpr int rows_wide() {
    constexpr int t = (1 << L) / 16, lo = t >= 64 ? 1 : 64 / t, cap = 4096 / (1 << L) < 8 ? 4096 / (1 << L) : 8;
    return lo > cap ? lo : cap;
}
template <int L>
constexpr int rows_narrow() {
    constexpr int t = (1 << L) / 16;
    return t >= 64 ? 1 : 64 / t;
}

// Block of rows of work-group b among g: XCD-major (see above).
__device__ __forceinline__ int row_block(int b, int g) { return (g & 7) ? b : (b & 7) * (g >> 3) + (b >> 3); }

// Lanes run over the RW rows of a work-group first (thread = j RW + rr), so
// that one load or store of a wave covers 64/RW consecutive elements of RW
// consecutive rows: whole 128-byte lines of a column block when RW = 8.  The
// rows' LDS spans start 16/RW 16-byte bank groups apart (lrow), so that the
// RW lanes with one j fall in different banks.
template <int LOG2N, int RW>
constexpr int lrow() {
    constexpr int base = (1 << LOG2N) + (1 << LOG2N) / 16, d = RW >= 16 ? 1 : 16 / RW;
    return RW == 1 ? base : base + (((d - base) % 16) + 16) % 16;
}
// p + byte_offset for a uniform p: a 32-bit per-lane offset (the arrays are
// below 4 GB), which the loads and stores take as such
__device__ __forceinline__ double2 *at(double2 *p, uint32_t byte_offset) {
    return reinterpret_cast<double2 *>(reinterpret_cast<char *>(p) + byte_offset);
}
__device__ __forceinline__ const double2 *at(const double2 *p, uint32_t byte_offset) {
    return reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(p) + byte_offset);
}

enum RowMode { kRowsFwd, kRowsMid, kRowsInv };

// Grid rows i (n = n_R points), per MODE (see above).  RW rows per
// work-group of RW n/16 threads.
template <int LOG2N, int RW, int MODE>
__global__ void __launch_bounds__(RW *(1 << LOG2N) / 16) __attribute__((amdgpu_waves_per_eu(2))) k_exact_rows(double2 *__restrict__ psi,
                                                                    const double2 *__restrict__ half,
                                                                    const double2 *__restrict__ tw,
                                                                    double2 *__restrict__ tmp, int nr) {
    constexpr int n = 1 << LOG2N, T = n / 16, LROW = lrow<LOG2N, RW>();
    __shared__ double2 lds[RW * LROW];
    const int rr = threadIdx.x % RW, j = threadIdx.x / RW;
    const int i0 = row_block(blockIdx.x, gridDim.x) * RW;
    double2 *row = lds + rr * LROW;
    double2 *p = psi + (size_t)i0 * n;          // rows i0 + rr of Psi: element (rr, k) at k + rr n
    const double2 *h = half + (size_t)i0 * n;
    double2 *t = tmp + i0;                      // columns i0 + rr of tmp [n_R][n_r]: element (rr, k) at k nr + rr
    auto rowel = [&](int m) { return (uint32_t)(((j + T * m) + rr * n) * sizeof(double2)); };
    auto colel = [&](int m) { return (uint32_t)(((size_t)(j + T * m) * nr + rr) * sizeof(double2)); };
    double2 v[16], hv[16];
    if constexpr (MODE == kRowsFwd) unroll<16>([&](auto m) { v[m.value] = *at(p, rowel(m.value)); });
    else unroll<16>([&](auto m) { v[m.value] = *at(t, colel(m.value)); });
    TwBase<LOG2N> tb;
    load_tw_base(tb, tw, j);
    auto load_half = [&] { unroll<16>([&](auto m) { hv[m.value] = *at(h, rowel(m.value)); }); };
    if constexpr (MODE == kRowsFwd) {
        load_half();
        unroll<16>([&](auto m) { v[m.value] = cmul(hv[m.value], v[m.value]); });
    } else {
        fft_row<LOG2N, true>(v, row, tw, tb, j, load_half);
        if constexpr (MODE == kRowsInv) {
            unroll<16>([&](auto m) { *at(p, rowel(m.value)) = cmul(hv[m.value], v[m.value]); });
            return;
        }
        unroll<16>([&](auto m) { v[m.value] = cmul(hv[m.value], cmul(hv[m.value], v[m.value])); });
    }
    fft_row<LOG2N, false>(v, row, tw, tb, j);
    unroll<16>([&](auto m) { *at(t, colel(m.value)) = v[m.value]; });
}

// Rows k_R of tmp (n = n_r points) -> IFFT_r(kin o FFT_r(row)), in place;
// kin = kin_R[k_R] kin_r[k_r].
template <int LOG2N, int RW>
__global__ void __launch_bounds__(RW *(1 << LOG2N) / 16) __attribute__((amdgpu_waves_per_eu(2))) k_exact_cols(
    double2 *__restrict__ tmp, const double2 *__restrict__ kin_r, const double2 *__restrict__ kin_R,
    const double2 *__restrict__ tw) {
    constexpr int n = 1 << LOG2N, T = n / 16, LROW = lrow<LOG2N, RW>();
    __shared__ double2 lds[RW * LROW];
    const int rr = threadIdx.x % RW, j = threadIdx.x / RW;
    const int c0 = row_block(blockIdx.x, gridDim.x) * RW, c = c0 + rr;
    double2 *row = lds + rr * LROW;
    double2 *q = tmp + (size_t)c0 * n;          // rows c0 + rr of tmp: element (rr, k) at k + rr n
    auto rowel = [&](int m) { return (uint32_t)(((j + T * m) + rr * n) * sizeof(double2)); };
    double2 v[16], kv[16];
    unroll<16>([&](auto m) { v[m.value] = *at(q, rowel(m.value)); });
    const double2 kR = kin_R[c];
    TwBase<LOG2N> tb;
    load_tw_base(tb, tw, j);
    fft_row<LOG2N, false>(v, row, tw, tb, j, [&] { unroll<16>([&](auto m) { kv[m.value] = kin_r[j + T * m.value]; }); });
    unroll<16>([&](auto m) { v[m.value] = cmul(cmul(kR, kv[m.value]), v[m.value]); });
    fft_row<LOG2N, true>(v, row, tw, tb, j);
    unroll<16>([&](auto m) { *at(q, rowel(m.value)) = v[m.value]; });
}

template <int L, int MODE>
void pass_rows(int nr, const ExactBufs &e, hipStream_t s) {
    constexpr int wide = rows_wide<L>(), narrow = rows_narrow<L>(), t = (1 << L) / 16;
    if (nr / wide >= 256 || wide == narrow)
        hipLaunchKernelGGL((k_exact_rows<L, wide, MODE>), dim3(nr / wide), dim3(wide * t), 0, s, e.psi, e.half, e.tw_R,
                           e.tmp, nr);
    else
        hipLaunchKernelGGL((k_exact_rows<L, narrow, MODE>), dim3(nr / narrow), dim3(narrow * t), 0, s, e.psi, e.half,
                           e.tw_R, e.tmp, nr);
}
template <int L>
void pass_rows_fwd(int nr, const ExactBufs &e, hipStream_t s) {
    pass_rows<L, kRowsFwd>(nr, e, s);
}
template <int L>
void pass_rows_mid(int nr, const ExactBufs &e, hipStream_t s) {
    pass_rows<L, kRowsMid>(nr, e, s);
}
template <int L>
void pass_rows_inv(int nr, const ExactBufs &e, hipStream_t s) {
    pass_rows<L, kRowsInv>(nr, e, s);
}
template <int L>
void pass_cols(int nR, const ExactBufs &e, hipStream_t s) {
    constexpr int wide = rows_wide<L>(), narrow = rows_narrow<L>(), t = (1 << L) / 16;
    if (nR / wide >= 256 || wide == narrow)
        hipLaunchKernelGGL((k_exact_cols<L, wide>), dim3(nR / wide), dim3(wide * t), 0, s, e.tmp, e.kin_r, e.kin_R, e.tw_r);
    else
        hipLaunchKernelGGL((k_exact_cols<L, narrow>), dim3(nR / narrow), dim3(narrow * t), 0, s, e.tmp, e.kin_r,
                           e.kin_R, e.tw_r);
}

// n = 2^lg for lg in [5, 12] (grid sizes 32 ... 4096, checked by the caller).
#define ICWF_EXACT_DISPATCH(fn, lg, ...)  \
    switch (lg) {                          \
    case 5: fn<5>(__VA_ARGS__); break;     \
    case 6: fn<6>(__VA_ARGS__); break;     \
    case 7: fn<7>(__VA_ARGS__); break;     \
    case 8: fn<8>(__VA_ARGS__); break;     \
    case 9: fn<9>(__VA_ARGS__); break;     \
    case 10: fn<10>(__VA_ARGS__); break;   \
    case 11: fn<11>(__VA_ARGS__); break;   \
    case 12: fn<12>(__VA_ARGS__); break;   \
    default: break;                        \
    }

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

void launch_exact_steps(int nr, int nR, const ExactBufs &e, int64_t nsteps, hipStream_t s) {
    if (nsteps <= 0) return;
    const int lr = log2i(nr), lR = log2i(nR);
    ICWF_EXACT_DISPATCH(pass_rows_fwd, lR, nr, e, s);
    for (int64_t k = 0; k < nsteps; ++k) {
        ICWF_EXACT_DISPATCH(pass_cols, lr, nR, e, s);
        if (k + 1 < nsteps) {
            ICWF_EXACT_DISPATCH(pass_rows_mid, lR, nr, e, s);
        } else {
            ICWF_EXACT_DISPATCH(pass_rows_inv, lR, nr, e, s);
        }
    }
}

}  // namespace icwf
