// Discretization (Section 2.1) and the dense on-the-fly product y = A x.
#include <cmath>
#include <mutex>

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
    CBD_LAUNCH(k_assemble, dim3(blocks), dim3(256), 0, s, d, n, grid, N, b, c, pts, diag,
                       w, rs, a_self, weight);
}

// y = A x on FP64 matrix cores.  A workgroup of kMvWaves waves owns
// kMvWaves * RB * 16 rows i (RB row blocks of 16 per wave) and up to 64
// right-hand sides (NB blocks of 16).  Sources j stream through LDS in tiles of
// kTJ points: coordinates, and w_j x_j stored [rhs][j] with a row stride of
// kTJ + 2 doubles, so that the staging writes and the B-operand reads both spread
// over the LDS banks.  Per K-step of 4 sources every lane generates one kernel
// value K(x_i - x_j) per row block on the VALU (lane l: i = l % 16, j = l / 16),
// which is the A operand of v_mfma_f64_16x16x4f64 for all NB right-hand-side
// blocks; the B operand is w_j x_j read from LDS (lane l: j = l / 16,
// rhs = l % 16).  Accumulator register v (v < 4) of lane l holds row 4 v + l / 16
// of column l % 16.  The diagonal term diag_i x_i is added at the end.
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMvThreads = 256;
constexpr int kMvWaves = kMvThreads / 64;
constexpr int kTJ = 64;                // sources per LDS tile
constexpr int kLdw = kTJ + 2;          // LDS row stride of the [rhs][j] tile (doubles)
constexpr int kLogBits = 11;
constexpr int kLogTab = 1 << kLogBits;

// 2D kernel value from r^2: K = -(1/2pi) log r = c log r^2, c = -1/(4 pi).
// Table-driven logarithm (after Tang, ACM TOMS 15(2), 1989), with the constant c
// folded into the table and the polynomial: r^2 = 2^e m, m in [1/2, 1) (frexp);
// the top 11 fraction bits of m select the interval [1/2 + j/4096, 1/2 + (j+1)/4096)
// and its midpoint F_j, so u = m/F_j - 1 lies in (-2^-12, 2^-12);
// c log r^2 = e (c ln2) + c log F_j + c log1p(u), with log1p(u) by its Taylor series
// to u^3 (alternating, so the truncation is below u^4/4 < 9e-16, i.e. 7e-17 absolute
// after the factor c).  tab[2j] = c log F_j and tab[2j+1] = 1/F_j, rounded from long
// double on the host.  r^2 = 0 (the pair i = j) gives e = 0, m = 0 and a finite
// value, which the product's epilogue removes again.
__device__ __forceinline__ double klog_r2(double x, const double* __restrict__ tab) {
    constexpr double c = -kInv4Pi;
    constexpr double cln2 = -kInv4Pi * 0.69314718055994530942;
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(x) >> 32);
    // the high word holds the top 20 fraction bits; entry j is 16 bytes
    const unsigned off = (hi >> (16 - kLogBits)) & ((kLogTab - 1) << 4);
    const double2 t = *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(tab) + off);
    const double u = fma(m, t.y, -1.0);
    double p = c / 3.0;
    p = fma(p, u, -c / 2.0);
    p = fma(p, u, c);
    return fma((double)e, cln2, fma(p, u, t.x));
}

template <int D>
__device__ __forceinline__ double kernel_r2(double r2, const double* __restrict__ tab) {
    if constexpr (D == 2)
        return klog_r2(r2, tab);
    else
        return kInv4Pi * rsqrt(r2);
}

// LDS of the product, small arrays first so that every access keeps a 16-bit immediate
// offset; the log table only in 2D
template <int D>
struct MvShared {
    double sxj[D][kTJ];
    double swx[64 * kLdw];
    alignas(16) double stab[D == 2 ? 2 * kLogTab : 2];
};

constexpr int kSR = kMvThreads / kTJ;  // staging threads per source
static_assert(kMvThreads % kTJ == 0 && 64 % kSR == 0, "staging layout");

template <int D, int NB, int kRB>
__global__ __launch_bounds__(kMvThreads) void k_matvec(ProblemView P, int nrhs,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y,
                                                       const double* __restrict__ logtab) {
    __shared__ MvShared<D> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long N = P.N;
    const int r0 = blockIdx.y * 64;
    const long ibase = (long)blockIdx.x * (kMvWaves * kRB * 16) + wave * (kRB * 16);
    const int li = lane & 15, lk = lane >> 4;
    if (D == 2)
        for (int e = tid; e < 2 * kLogTab; e += kMvThreads) sh.stab[e] = logtab[e];

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
        // stage the tile: coordinates and w_j x_j (zero for padding sources / columns);
        // thread t stages source j0 + t % kTJ for right-hand sides t / kTJ + kSR q.
        // The loads use clamped, always valid indices and are masked afterwards, so
        // all of them are in flight at once.
        {
            const int sj = tid % kTJ, sr = tid / kTJ;
            const long j = j0 + sj;
            const bool jin = j < N;
            const long jc = jin ? j : N - 1;
            const double wj = jin ? P.w[jc] : 0.0;
            if (sr < D) sh.sxj[sr][sj] = jin ? P.pts[sr * N + jc] : 8.0 + sr;
            constexpr int kQ = NB * 16 / kSR;
            double v[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int rr = min(r0 + sr + kSR * q, nrhs - 1);
                v[q] = x[(long)rr * N + jc];
            }
#pragma unroll
            for (int q = 0; q < kQ; ++q) {
                const int r = sr + kSR * q;
                sh.swx[r * kLdw + sj] = (r0 + r < nrhs) ? wj * v[q] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int ks = 0; ks < kTJ / 4; ++ks) {
            const int jj = ks * 4 + lk;
            double xj[D];
#pragma unroll
            for (int t = 0; t < D; ++t) xj[t] = sh.sxj[t][jj];
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
                    // the pair i == j enters with the finite value at r^2 = 0; the epilogue removes it
                    a[rb] = kernel_r2<D>(r2, sh.stab);
                } else {
                    const double kv = kernel_r2<D>(r2, sh.stab);
                    a[rb] = (j0 + jj == irow[rb]) ? 0.0 : kv;
                }
            }
            double b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = sh.swx[(nb * 16 + li) * kLdw + jj];
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
            // 2D: remove the self pair, which entered with the value at r^2 = 0
            const double selfw = (D == 2) ? kernel_r2<D>(0.0, sh.stab) * P.w[i] : 0.0;
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

// The same product on the 2D uniform grid, with the entries taken from a table.
// Grid points are g = j1 + n j2 and x_i - x_j = spacing (j(i) - j(j)), so an entry
// depends only on the offset (Delta1, Delta2) (the translation invariance the FFT form
// uses as well).  A workgroup's rows are R = 16 kW kRB consecutive points of one grid
// line, and a source tile is T consecutive points of one line (T = 64 with 4 waves,
// 128 with 8; n a multiple of R and T); the pair then meets only R + T - 1 offsets:
// Delta2 fixed and Delta1 = (i1_0 - j1_0) + delta - (T - 1) for delta = row offset -
// source offset + T - 1.  Each tile's R + T - 1 kernel values are evaluated once into
// LDS (the pair i = j gets 0: the diagonal is added at the end), and a lane's A
// operand is one LDS read at delta.  Products, summation order and epilogue are those
// of k_matvec.
template <int kRows, int kT>
struct MvGridShared {
    double swx[64 * (kT + 2)];
    double ktab[kRows + kT];
};
constexpr int grid_tile(int waves) { return waves == 8 ? 128 : kTJ; }

template <int NB, int kRB, int kW>
__global__ __launch_bounds__(64 * kW) void k_matvec_grid2(ProblemView P, int nrhs,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ y) {
    constexpr int kThr = 64 * kW;             // kW waves per workgroup
    constexpr int kR = kW * kRB * 16;         // rows per workgroup
    constexpr int kT = grid_tile(kW);         // sources per tile
    constexpr int kLd = kT + 2;               // LDS row stride of the [rhs][j] tile
    constexpr int kSRw = kThr / kT;           // staging threads per source
    __shared__ MvGridShared<kR, kT> shb[2];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long N = P.N;
    const int n = P.n;
    const int r0 = blockIdx.y * 64;
    const long iw = (long)blockIdx.x * kR;            // first row of the workgroup
    const long ibase = iw + wave * (kRB * 16);
    const int li = lane & 15, lk = lane >> 4;
    const long i2 = iw / n, i1_0 = iw % n;
    const double sp2 = P.spacing * P.spacing;
    // per-lane table position of row li, source lk at K-step 0 and row block 0
    const int d0 = wave * (kRB * 16) + li - lk + (kT - 1);

    v4d acc[kRB][NB];
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[rb][nb] = v4d{0.0, 0.0, 0.0, 0.0};

    // Software pipeline over source tiles, two LDS buffers: during tile t's products
    // the next tile's staging (x, w and the offsets' kernel values, fetched into
    // registers one tile earlier) is written to the other buffer, and the tile after
    // that is fetched; one barrier per tile.
    const int sj = tid % kT, sr = tid / kT;
    constexpr int kQ = NB * 16 / kSRw;
    static_assert(kQ * kSRw == NB * 16, "staging layout");
    constexpr int kKT = (kR + kT - 1 + kThr - 1) / kThr;   // table entries per thread
    double v[kQ], wj, kt[kKT];
    auto fetch = [&](long j0) {
        const long j = j0 + sj;
        wj = P.w[j];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int rr = min(r0 + sr + kSRw * q, nrhs - 1);
            v[q] = x[(long)rr * N + j];
        }
        const long d2 = i2 - j0 / n;
        const long d1base = i1_0 - (j0 % n) - (kT - 1);
#pragma unroll
        for (int u = 0; u < kKT; ++u) {
            const int e = tid + u * kThr;
            const long d1 = d1base + e;
            const long q = d1 * d1 + d2 * d2;
            kt[u] = (e >= kR + kT - 1 || q == 0) ? 0.0 : laplace_from_r2<2>((double)q * sp2);
        }
    };
    auto stage = [&](MvGridShared<kR, kT>& sh) {
#pragma unroll
        for (int u = 0; u < kKT; ++u) {
            const int e = tid + u * kThr;
            if (e < kR + kT - 1) sh.ktab[e] = kt[u];
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const int r = sr + kSRw * q;
            sh.swx[r * kLd + sj] = (r0 + r < nrhs) ? wj * v[q] : 0.0;
        }
    };
    fetch(0);
    stage(shb[0]);
    if (kT < N) fetch(kT);
    __syncthreads();
    int cur = 0;
    for (long j0 = 0; j0 < N; j0 += kT) {
        if (j0 + kT < N) stage(shb[cur ^ 1]);
        if (j0 + 2 * kT < N) fetch(j0 + 2 * kT);
        const MvGridShared<kR, kT>& sh = shb[cur];
#pragma unroll 1
        for (int ks = 0; ks < kT / 4; ++ks) {
            const int jj = ks * 4 + lk;
            const double* ta = sh.ktab + (d0 - ks * 4);
            double a[kRB];
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb) a[rb] = ta[rb * 16];
            double b[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) b[nb] = sh.swx[(nb * 16 + li) * kLd + jj];
#pragma unroll
            for (int rb = 0; rb < kRB; ++rb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[rb][nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[nb], acc[rb][nb], 0, 0, 0);
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int rb = 0; rb < kRB; ++rb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long i = ibase + rb * 16 + 4 * v + lk;
            const double bi = P.rs[i], di = P.diag[i];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int r = r0 + nb * 16 + li;
                if (r < nrhs) {
                    const long o = (long)r * N + i;
                    y[o] = bi * acc[rb][nb][v] + di * x[o];
                }
            }
        }
    }
}

// One right-hand side on the 2D grid: grid lines take the place of the right-hand
// sides in the MFMA columns.  Output line j2 receives, for every line offset Delta2,
// the Toeplitz block T_Delta2 (entries K(spacing |(Delta1, Delta2)|)) times source line
// j2 - Delta2, so 16 output lines b .. b + 15 share the A operand T_Delta2 and take
// their B columns from 16 different source lines (zero where j2 - Delta2 leaves the
// grid).  A workgroup owns 64 rows of 16 lines and runs over Delta2 = b - (n - 1) ..
// b + 15 and source tiles of 64 points; A comes from the tile's table of 127 offsets as
// in k_matvec_grid2.  The next tile's x and w are loaded into registers while the
// current one is multiplied.  Every output sums its sources in ascending Delta2 and,
// within a line, ascending position.
struct MvLinesShared {
    double sb[16 * kLdw];
    double ktab[128];
};

__global__ __launch_bounds__(kMvThreads) void k_matvec_lines2(ProblemView P, const double* __restrict__ x,
                                                              double* __restrict__ y) {
    __shared__ MvLinesShared sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = P.n;
    const long a = (long)blockIdx.x * 64;          // first row (position in the line)
    const long b = (long)blockIdx.y * 16;          // first output line
    const int li = lane & 15, lk = lane >> 4;
    const double sp2 = P.spacing * P.spacing;
    const int d0 = wave * 16 + li - lk + 63;
    const int ntile = n / kTJ;
    const long dlo = b - (n - 1), dhi = b + 15;
    const long niter = (dhi - dlo + 1) * ntile;
    // staging role: line column c = tid / 16, positions jj = (tid % 16) + 16 q
    const int sc = tid >> 4, sj = tid & 15;
    double xv[4], wv[4];
    auto load = [&](long it) {
        const long d2 = dlo + it / ntile;
        const long t0 = (it % ntile) * kTJ;
        const long src = b + sc - d2;                // source line of column sc
        const bool in = src >= 0 && src < n;
        const long base = (in ? src : 0) * (long)n + t0 + sj;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xv[q] = in ? x[base + 16 * q] : 0.0;
            wv[q] = in ? P.w[base + 16 * q] : 0.0;
        }
    };
    v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
    load(0);
    for (long it = 0; it < niter; ++it) {
        const long d2 = dlo + it / ntile;
        const long t0 = (it % ntile) * kTJ;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) sh.sb[sc * kLdw + sj + 16 * q] = wv[q] * xv[q];
        if (tid < 127) {
            const long d1 = a - t0 - 63 + tid;
            const long qd = d1 * d1 + d2 * d2;
            sh.ktab[tid] = qd == 0 ? 0.0 : laplace_from_r2<2>((double)qd * sp2);
        }
        if (it + 1 < niter) load(it + 1);
        __syncthreads();
#pragma unroll 4
        for (int ks = 0; ks < kTJ / 4; ++ks) {
            const double av = sh.ktab[d0 - 4 * ks];
            const double bv = sh.sb[li * kLdw + 4 * ks + lk];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
    }
    // register v of lane l: row 4 v + l / 16 of the wave's 16 rows, line b + l % 16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const long i = (b + li) * (long)n + a + wave * 16 + 4 * v + lk;
        y[i] = P.rs[i] * acc[v] + P.diag[i] * x[i];
    }
}

// c log F_j and 1/F_j (F_j = (1 + (j + 1/2)/2048)/2, c = -1/(4 pi)): a device symbol,
// filled once per device; host code passes its device address (hipGetSymbolAddress).
__device__ __align__(256) double g_logtab[2 * kLogTab];

static const double* log_table() {
    static std::mutex mx;
    static const double* addr[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(mx);
    if (!addr[dev]) {
        static double h[2 * kLogTab];
        const long double c = -0.25L / 3.141592653589793238462643383279502884L;
        for (int j = 0; j < kLogTab; ++j) {
            const long double F = 0.5L + ((long double)j + 0.5L) / (2.0L * kLogTab);
            h[2 * j] = (double)(c * std::log(F));
            h[2 * j + 1] = (double)(1.0L / F);
        }
        void* d = nullptr;
        if (hipGetSymbolAddress(&d, HIP_SYMBOL(g_logtab)) != hipSuccess || !d) return nullptr;
        if (hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        addr[dev] = (const double*)d;
    }
    return addr[dev];
}

bool matvec_prepare() { return log_table() != nullptr; }

// Tile shapes: rb row blocks of 16 per wave, with 4 waves per workgroup for rb = 1, 2, 4
// and 8 waves (the table form only) for rb = 8 + 1, 8 + 2, 8 + 4.
static int shape_rb(int rb) { return rb & 7; }
static int shape_waves(int rb) { return rb >= 8 ? 8 : kMvWaves; }

// The table form needs whole grid lines per workgroup and per source tile.
static bool matvec_grid_form(const ProblemView& P, int rb) {
    return P.d == 2 && P.n % matvec_rows_per_block(rb) == 0 && P.n % grid_tile(shape_waves(rb)) == 0;
}

template <int D, int NB, int RB>
static void matvec_launch(const ProblemView& P, int nrhs, const double* x, double* y, int max_blocks,
                          hipStream_t s) {
    const int rows = matvec_rows_per_block(RB);
    int blocks = (int)((P.N + rows - 1) / rows);
    if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
    dim3 grid(blocks, (nrhs + 63) / 64);
    if (D == 2 && matvec_grid_form(P, RB)) {
        if constexpr (RB >= 8)
            CBD_LAUNCH((k_matvec_grid2<NB, RB & 7, 8>), grid, dim3(512), 0, s, P, nrhs, x, y);
        else
            CBD_LAUNCH((k_matvec_grid2<NB, RB, kMvWaves>), grid, dim3(kMvThreads), 0, s, P, nrhs, x, y);
        return;
    }
    CBD_LAUNCH((k_matvec<D, NB, (RB & 7)>), grid, dim3(kMvThreads), 0, s, P, nrhs, x, y, log_table());
}

template <int D, int NB>
static void matvec_rb(const ProblemView& P, int nrhs, const double* x, double* y, int rb, int max_blocks,
                      hipStream_t s) {
    switch (rb) {
        case 1: matvec_launch<D, NB, 1>(P, nrhs, x, y, max_blocks, s); break;
        case 2: matvec_launch<D, NB, 2>(P, nrhs, x, y, max_blocks, s); break;
        case 8 + 1: matvec_launch<D, NB, 8 + 1>(P, nrhs, x, y, max_blocks, s); break;
        case 8 + 2: matvec_launch<D, NB, 8 + 2>(P, nrhs, x, y, max_blocks, s); break;
        case 8 + 4: matvec_launch<D, NB, 8 + 4>(P, nrhs, x, y, max_blocks, s); break;
        default: matvec_launch<D, NB, 4>(P, nrhs, x, y, max_blocks, s); break;
    }
}

int matvec_rows_per_block(int rb) { return shape_waves(rb) * 16 * shape_rb(rb); }

// Right-hand-side blocks of 16 handled per launch column (the grid's y covers groups of 64).
int matvec_nb(int nrhs) { return nrhs > 64 ? 4 : (nrhs + 15) / 16; }

// Default row blocks per wave: 4 while the accumulators (RB * NB * 4 doubles)
// leave room for three waves per SIMD, else 2.
int matvec_default_rb(int nb) { return nb <= 2 ? 4 : 2; }

void launch_matvec(const ProblemView& P, int nrhs, const double* x, double* y, int rb, int max_blocks,
                   hipStream_t s) {
    if (nrhs == 1 && P.d == 2 && P.n % kTJ == 0 && max_blocks <= 0) {
        // one right-hand side: grid lines fill the MFMA columns
        CBD_LAUNCH(k_matvec_lines2, dim3(P.n / 64, P.n / 16), dim3(kMvThreads), 0, s, P, x, y);
        return;
    }
    const int nb = matvec_nb(nrhs);
    if (rb <= 0) rb = matvec_default_rb(nb);
    // 2D grids whose lines hold whole workgroups use the table form: the largest row
    // block count up to rb that fits
    // (shapes of 8 waves exist in the table form only)
    if (P.d != 2 || !matvec_grid_form(P, rb)) rb = shape_rb(rb);
    if (P.d == 2 && !matvec_grid_form(P, rb)) {
        int r = rb;
        while (r > 1 && !matvec_grid_form(P, r)) r /= 2;
        if (matvec_grid_form(P, r)) rb = r;
    }
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
