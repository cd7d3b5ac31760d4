// Discretization (Section 2.1) and the dense on-the-fly product y = A x.
#include <cmath>

#include "internal.h"

namespace cbd {

__global__ void k_assemble(int d, int n, int grid, long N, const double* __restrict__ b,
                           const double* __restrict__ c, double* __restrict__ pts,
                           double* __restrict__ diag, double* __restrict__ w,
                           double* __restrict__ rs, double a_self, double weight) {
    long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    long rem = g;
    for (int t = 0; t < d; ++t) {
        long j = rem % n;
        rem /= n;
        pts[t * N + g] = (grid == 0) ? ((double)j + 0.5) / (double)n : (double)j / (double)(n - 1);
    }
    double bi = b ? b[g] : 1.0;
    double ci = c ? c[g] : 1.0;
    rs[g] = bi;
    w[g] = weight * ci;
    diag[g] = bi * ci * a_self;
}

void launch_assemble(int d, int n, int grid, const double* b, const double* c, double* pts,
                     double* diag, double* w, double* rs, double a_self, double weight,
                     hipStream_t s) {
    long N = 1;
    for (int t = 0; t < d; ++t) N *= n;
    int blocks = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_assemble, dim3(blocks), dim3(256), 0, s, d, n, grid, N, b, c, pts, diag,
                       w, rs, a_self, weight);
}

// y = A x on FP64 matrix cores.  A 256-thread workgroup owns 256 rows i (4 waves
// x RB = 4 row blocks of 16) and up to 64 right-hand sides (NB blocks of 16).
// Sources j stream through LDS in tiles of kTJ points (coordinates and w_j x_j,
// stored [j][rhs]).  Per K-step of 4 sources every lane generates one kernel
// value K(x_i - x_j) per row block on the VALU (lane l: i = l % 16, j = l / 16),
// which is the A operand of v_mfma_f64_16x16x4f64 for all NB right-hand-side
// blocks; the B operand is w_j x_j read from LDS (lane l: j = l / 16,
// rhs = l % 16).  Accumulator register v (v < 4) of lane l holds row 4 v + l / 16
// of column l % 16.  The diagonal term diag_i x_i is added at the end.
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMvThreads = 256;
constexpr int kTJ = 64;
constexpr int kLogTab = 128;
// 2D self pair: r^2 is clamped to 2^-1000 (K = 55.1...), removed exactly in the epilogue
constexpr double kSelfR2 = 0x1p-1000;

// Table-driven natural logarithm (Tang, ACM TOMS 15(2), 1989) for positive normal
// x: x = 2^e m, m in [1, 2); F = 1 + j/128 from the top 7 mantissa bits (so
// m - F is exact and u = (m - F)/F is in [0, 1/128)); log x = e ln2 + log F +
// log1p(u), log1p by its Taylor series to u^8 (truncation < 2e-18 relative).
// tab[2j] = log F_j, tab[2j+1] = 1/F_j (from the host's libm).
__device__ __forceinline__ double log_tab(double x, const double* __restrict__ tab) {
    constexpr double kLn2Hi = 0x1.62e42fp-1;
    constexpr double kLn2Lo = 0x1.df473de6af279p-26;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    const unsigned hi = (unsigned)(bits >> 32), lo = (unsigned)bits;
    const int e = (int)(hi >> 20) - 1023;
    const unsigned mhi = (hi & 0x000FFFFFu) | 0x3FF00000u;
    const double m = __longlong_as_double((long long)(((unsigned long long)mhi << 32) | lo));
    const double F = __longlong_as_double((long long)((unsigned long long)(mhi & 0xFFFFE000u) << 32));
    const int j = (mhi >> 13) & (kLogTab - 1);
    const double u = (m - F) * tab[2 * j + 1];
    double p = -1.0 / 8.0;
    p = fma(p, u, 1.0 / 7.0);
    p = fma(p, u, -1.0 / 6.0);
    p = fma(p, u, 1.0 / 5.0);
    p = fma(p, u, -1.0 / 4.0);
    p = fma(p, u, 1.0 / 3.0);
    p = fma(p, u, -1.0 / 2.0);
    p = fma(p * u, u, u);                                  // log1p(u)
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, tab[2 * j]) + p);
}

template <int D>
__device__ __forceinline__ double kernel_r2(double r2, const double* __restrict__ tab) {
    if constexpr (D == 2)
        return -0.5 * kInv2Pi * log_tab(r2, tab);
    else
        return kInv4Pi * rsqrt(r2);
}                // sources per LDS tile
constexpr int kLdw = 66;               // LDS row stride of the [j][rhs] tile (doubles)

template <int D, int NB, int kRB>
__global__ __launch_bounds__(kMvThreads) void k_matvec(ProblemView P, int nrhs,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y,
                                                       const double* __restrict__ logtab) {
    __shared__ double sxj[D][kTJ];
    __shared__ double swx[kTJ * kLdw];
    __shared__ double stab[2 * kLogTab];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long N = P.N;
    const int r0 = blockIdx.y * 64;
    const long ibase = (long)blockIdx.x * (4 * kRB * 16) + wave * (kRB * 16);
    const int li = lane & 15, lk = lane >> 4;
    if (D == 2)
        for (int e = tid; e < 2 * kLogTab; e += kMvThreads) stab[e] = logtab[e];

    double xi[kRB][D];
    long irow[kRB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
        irow[rb] = ibase + rb * 16 + li;
#pragma unroll
        for (int t = 0; t < D; ++t)
            xi[rb][t] = irow[rb] < N ? P.pts[t * N + irow[rb]] : 4.0 + t;   // padding rows: far away
    }
    v4d acc[kRB][NB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = v4d{0.0, 0.0, 0.0, 0.0};

    for (long j0 = 0; j0 < N; j0 += kTJ) {
        __syncthreads();
        // stage the tile: coordinates and w_j x_j (zero for padding sources / columns)
        for (int e = tid; e < D * kTJ; e += kMvThreads) {
            const int t = e / kTJ, jj = e % kTJ;
            const long j = j0 + jj;
            sxj[t][jj] = j < N ? P.pts[t * N + j] : 8.0 + t;
        }
        for (int e = tid; e < NB * 16 * kTJ; e += kMvThreads) {
            const int r = e / kTJ, jj = e % kTJ;
            const long j = j0 + jj;
            double v = 0.0;
            if (j < N && r0 + r < nrhs) v = P.w[j] * x[(long)(r0 + r) * N + j];
            swx[jj * kLdw + r] = v;
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < kTJ / 4; ++ks) {
            const int jj = ks * 4 + lk;
            double xj[D];
#pragma unroll
            for (int t = 0; t < D; ++t) xj[t] = sxj[t][jj];
            double a[kRB];
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb) {
                double r2 = 0.0;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const double dx = xi[rb][t] - xj[t];
                    r2 = fma(dx, dx, r2);
                }
                if constexpr (D == 2) {
                    // the pair i == j enters as K(kSelfR2); the epilogue removes it
                    a[rb] = kernel_r2<D>(fmax(r2, kSelfR2), stab);
                } else {
                    const double kv = kernel_r2<D>(r2, stab);
                    a[rb] = (j0 + jj == irow[rb]) ? 0.0 : kv;
                }
            }
            double b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = swx[jj * kLdw + nb * 16 + li];
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[rb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[nb], acc[rb][nb], 0, 0, 0);
        }
    }
    // epilogue: register v of lane l holds row 4*v + l/16 of column l%16
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long i = ibase + rb * 16 + 4 * v + lk;
            if (i >= N) continue;
            const double bi = P.rs[i], di = P.diag[i];
            // 2D: remove the self pair, which entered as K(kSelfR2) w_i x_i
            const double selfw = (D == 2) ? kernel_r2<D>(kSelfR2, stab) * P.w[i] : 0.0;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int r = r0 + nb * 16 + li;
                if (r < nrhs) {
                    const long o = (long)r * N + i;
                    const double xo = x[o];
                    y[o] = bi * (acc[rb][nb][v] - selfw * xo) + di * xo;
                }
            }
        }
    }
}

// log F_j and 1/F_j, F_j = 1 + j/128, uploaded once per device.
static const double* log_table() {
    static double* dtab[64] = {nullptr};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64) return nullptr;
    if (!dtab[dev]) {
        double h[2 * kLogTab];
        for (int j = 0; j < kLogTab; ++j) {
            const double F = 1.0 + j / 128.0;
            h[2 * j] = std::log(F);
            h[2 * j + 1] = 1.0 / F;
        }
        double* d = nullptr;
        if (hipMalloc(&d, sizeof(h)) != hipSuccess) return nullptr;
        if (hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        dtab[dev] = d;
    }
    return dtab[dev];
}

bool matvec_prepare() { return log_table() != nullptr; }

template <int D, int NB, int RB>
static void matvec_launch(const ProblemView& P, int nrhs, const double* x, double* y, int max_blocks,
                          hipStream_t s) {
    const int rows = 4 * RB * 16;
    int blocks = (int)((P.N + rows - 1) / rows);
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    dim3 grid(blocks, (nrhs + 63) / 64);
    hipLaunchKernelGGL((k_matvec<D, NB, RB>), grid, dim3(kMvThreads), 0, s, P, nrhs, x, y, log_table());
}

template <int D, int NB>
static void matvec_rb(const ProblemView& P, int nrhs, const double* x, double* y, int rb, int max_blocks,
                      hipStream_t s) {
    switch (rb) {
        case 1: matvec_launch<D, NB, 1>(P, nrhs, x, y, max_blocks, s); break;
        case 2: matvec_launch<D, NB, 2>(P, nrhs, x, y, max_blocks, s); break;
        default: matvec_launch<D, NB, 4>(P, nrhs, x, y, max_blocks, s); break;
    }
}

// Right-hand-side blocks of 16 handled per launch column (the grid's y covers groups of 64).
int matvec_nb(int nrhs) { return nrhs > 64 ? 4 : (nrhs + 15) / 16; }

// Default row blocks per wave: 4 while the accumulators (RB * NB * 4 doubles)
// leave room for three waves per SIMD, else 2.
int matvec_default_rb(int nb) { return nb <= 2 ? 4 : 2; }

void launch_matvec(const ProblemView& P, int nrhs, const double* x, double* y, int rb, int max_blocks,
                   hipStream_t s) {
    const int nb = matvec_nb(nrhs);
    if (rb <= 0) rb = matvec_default_rb(nb);
    if (P.d == 2) {
        switch (nb) {
            case 1: matvec_rb<2, 1>(P, nrhs, x, y, rb, max_blocks, s); break;
            case 2: matvec_rb<2, 2>(P, nrhs, x, y, rb, max_blocks, s); break;
            case 3: matvec_rb<2, 3>(P, nrhs, x, y, rb, max_blocks, s); break;
            default: matvec_rb<2, 4>(P, nrhs, x, y, rb, max_blocks, s); break;
        }
    } else {
        switch (nb) {
            case 1: matvec_rb<3, 1>(P, nrhs, x, y, rb, max_blocks, s); break;
            case 2: matvec_rb<3, 2>(P, nrhs, x, y, rb, max_blocks, s); break;
            case 3: matvec_rb<3, 3>(P, nrhs, x, y, rb, max_blocks, s); break;
            default: matvec_rb<3, 4>(P, nrhs, x, y, rb, max_blocks, s); break;
        }
    }
}

}  // namespace cbd
