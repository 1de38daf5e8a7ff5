// Propagation of the full two-dimensional wavefunction Psi(r_i, R_j) (Eq. 1
// with the Hamiltonian of Eq. 2 on the product grid), by the same Strang
// split operator the conditional wavefunctions use, in two dimensions:
//
//     Psi <- e^{-i W dt/2} IFFT2[ e^{-i (k_r^2/2m_r + k_R^2/2m_R) dt} FFT2[ e^{-i W dt/2} Psi ] ].
//
// This is the reference the ansatz of Eq. 7 converges to as N grows; it
// stores n_r n_R values where the method stores N (n_r + n_R).
//
// Three passes per step, one work-group per grid row (n/4 threads, 64 to
// 1024), each row transformed
// in LDS by a radix-4 Stockham FFT (autosort: no bit reversal):
//   1. rows i of Psi [n_r][n_R]: multiply by the half-step potential phase,
//      FFT along R, write transposed into tmp [n_R][n_r];
//   2. rows k_R of tmp: FFT along r, multiply by the kinetic phase (which
//      carries the 1/(n_r n_R) of the inverse transform), inverse FFT along r,
//      write transposed back into Psi;
//   3. rows i of Psi: inverse FFT along R, multiply by the half-step phase.
// The transposed writes are strided; the whole state is 2 MB at 512 x 256
// and 32 MB at 4096 x 512, so it stays in the caches between passes.

#include <hip/hip_runtime.h>

#include "icwf_device.hpp"
#include "icwf_plan.hpp"

namespace icwf {
namespace {

// Threads per work-group for n = 2^L points: one radix-4 butterfly each
// (n / 4), at least one wave and at most 1024.
template <int L>
constexpr int exact_threads() {
    return (1 << L) / 4 < 64 ? 64 : ((1 << L) / 4 > 1024 ? 1024 : (1 << L) / 4);
}

// In-LDS FFT of n = 2^LOG2N points, starting in a, unscaled in both
// directions: Stockham autosort, radix 4 (one radix-2 pass first when LOG2N
// is odd).  A radix-4 pass with Ns points per finished sub-transform combines
// four of them: butterfly j reads a[j + r n/4] (r < 4), multiplies element r
// by e^{-/+ 2 pi i r (j mod Ns) / (4 Ns)}, takes the 4-point DFT and writes
// output s to b[(j div Ns) 4 Ns + j mod Ns + s Ns].  tw[m] = e^{-2 pi i m / n},
// m < n.  Returns the buffer holding the result; every thread has passed a
// barrier after the last write.
template <int LOG2N, int NT = exact_threads<LOG2N>()>
__device__ double2 *lds_fft(double2 *a, double2 *b, const double2 *__restrict__ tw, bool inverse,
                            int tid = threadIdx.x) {
    constexpr int n = 1 << LOG2N, q = n / 4, nt = NT;
    int ns = 1;
    if (LOG2N & 1) {                 // Ns = 1: no twiddles
        for (int j = tid; j < n / 2; j += nt) {
            const double2 v0 = a[j], v1 = a[j + n / 2];
            b[2 * j] = cadd(v0, v1);
            b[2 * j + 1] = csub(v0, v1);
        }
        __syncthreads();
        double2 *t = a;
        a = b;
        b = t;
        ns = 2;
    }
    for (; ns < n; ns <<= 2) {
        const int stride = q / ns;   // n / (4 Ns)
        for (int j = tid; j < q; j += nt) {
            const int k = j & (ns - 1);
            double2 w1 = tw[k * stride], w2 = tw[2 * k * stride], w3 = tw[3 * k * stride];
            if (inverse) {
                w1.y = -w1.y;
                w2.y = -w2.y;
                w3.y = -w3.y;
            }
            const double2 v0 = a[j], v1 = cmul(a[j + q], w1), v2 = cmul(a[j + 2 * q], w2),
                          v3 = cmul(a[j + 3 * q], w3);
            const double2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), d = csub(v1, v3);
            // -i d (forward) or +i d (inverse)
            const double2 a3 = inverse ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
            const int o = ((j - k) << 2) + k;
            b[o] = cadd(a0, a2);
            b[o + ns] = cadd(a1, a3);
            b[o + 2 * ns] = csub(a0, a2);
            b[o + 3 * ns] = csub(a1, a3);
        }
        __syncthreads();
        double2 *t = a;
        a = b;
        b = t;
    }
    return a;
}

// Pass 1: rows i of psi (n = n_R points) -> FFT_R(half_i o psi_i), stored as
// columns i of tmp [n_R][n_r].  A work-group takes fwd_rows<LOG2N> rows (a
// group of n/4 threads per row), so that each column of tmp receives that
// many consecutive values at once: up to a whole 128-byte line per write.
template <int L>
constexpr int fwd_rows() {
    return (1 << L) * 8 <= 4096 ? 8 : 4096 / (1 << L);     // <= 128 KB of LDS
}
template <int L>
constexpr int fwd_group() {
    return (1 << L) / 4;
}
template <int LOG2N>
__global__ void __launch_bounds__(fwd_rows<LOG2N>() * fwd_group<LOG2N>()) k_exact_rows_fwd(
    const double2 *__restrict__ psi, const double2 *__restrict__ half, const double2 *__restrict__ tw,
    double2 *__restrict__ tmp, int nr) {
    constexpr int n = 1 << LOG2N, RW = fwd_rows<LOG2N>(), G = fwd_group<LOG2N>(), nt = RW * G;
    __shared__ double2 buf[2][RW][n];
    const int r = threadIdx.x / G, tid = threadIdx.x - r * G;
    const size_t i0 = (size_t)blockIdx.x * RW;
    for (int e = threadIdx.x; e < RW * n; e += nt) {
        const int rr = e / n, j = e - rr * n;
        const size_t g = (i0 + rr) * n + j;
        buf[0][rr][j] = cmul(half[g], psi[g]);
    }
    __syncthreads();
    const double2 *res = lds_fft<LOG2N, G>(buf[0][r], buf[1][r], tw, false, tid);
    // every row's result sits in the same buffer (the passes are the same)
    const int sel = (res == buf[0][r]) ? 0 : 1;
    for (int e = threadIdx.x; e < RW * n; e += nt) {
        const int k = e / RW, rr = e - k * RW;
        tmp[(size_t)k * nr + i0 + rr] = buf[sel][rr][k];
    }
}

// Pass 2: row k_R of tmp (n = n_r points) -> IFFT_r(kin o FFT_r(row)), stored
// as column k_R of psi [n_r][n_R].
template <int LOG2N>
__global__ void __launch_bounds__(exact_threads<LOG2N>()) k_exact_cols(const double2 *__restrict__ tmp,
                                                              const double2 *__restrict__ kinT,
                                                              const double2 *__restrict__ tw,
                                                              double2 *__restrict__ psi, int nR) {
    constexpr int n = 1 << LOG2N, nt = exact_threads<LOG2N>();
    __shared__ double2 buf[2][n];
    const size_t row = (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += nt) buf[0][i] = tmp[row + i];
    __syncthreads();
    double2 *f = lds_fft<LOG2N>(buf[0], buf[1], tw, false);
    double2 *g = (f == buf[0]) ? buf[1] : buf[0];
    for (int k = threadIdx.x; k < n; k += nt) f[k] = cmul(kinT[row + k], f[k]);
    __syncthreads();
    const double2 *res = lds_fft<LOG2N>(f, g, tw, true);
    for (int i = threadIdx.x; i < n; i += nt) psi[(size_t)i * nR + blockIdx.x] = res[i];
}

// Pass 3: row i of psi (n = n_R points) -> half_i o IFFT_R(psi_i), in place.
template <int LOG2N>
__global__ void __launch_bounds__(exact_threads<LOG2N>()) k_exact_rows_inv(double2 *__restrict__ psi,
                                                                  const double2 *__restrict__ half,
                                                                  const double2 *__restrict__ tw) {
    constexpr int n = 1 << LOG2N, nt = exact_threads<LOG2N>();
    __shared__ double2 buf[2][n];
    const size_t row = (size_t)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += nt) buf[0][j] = psi[row + j];
    __syncthreads();
    const double2 *res = lds_fft<LOG2N>(buf[0], buf[1], tw, true);
    for (int j = threadIdx.x; j < n; j += nt) psi[row + j] = cmul(half[row + j], res[j]);
}

template <int L>
void pass_rows_fwd(int nr, const ExactBufs &e, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_rows_fwd<L>, dim3(nr / fwd_rows<L>()), dim3(fwd_rows<L>() * fwd_group<L>()), 0, s,
                       e.psi, e.half, e.tw_R, e.tmp, nr);
}
template <int L>
void pass_cols(int nR, const ExactBufs &e, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_cols<L>, dim3(nR), dim3(exact_threads<L>()), 0, s, e.tmp, e.kinT, e.tw_r, e.psi, nR);
}
template <int L>
void pass_rows_inv(int nr, const ExactBufs &e, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_rows_inv<L>, dim3(nr), dim3(exact_threads<L>()), 0, s, e.psi, e.half, e.tw_R);
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

void launch_exact_step(int nr, int nR, const ExactBufs &e, hipStream_t s) {
    const int lr = log2i(nr), lR = log2i(nR);
    ICWF_EXACT_DISPATCH(pass_rows_fwd, lR, nr, e, s);
    ICWF_EXACT_DISPATCH(pass_cols, lr, nR, e, s);
    ICWF_EXACT_DISPATCH(pass_rows_inv, lR, nr, e, s);
}

}  // namespace icwf
