// Discretization (Section 2.1) and the dense on-the-fly product y = A x.
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
constexpr int kTJ = 64;                // sources per LDS tile
constexpr int kLdw = 66;               // LDS row stride of the [j][rhs] tile (doubles)

template <int D, int NB, int kRB>
__global__ __launch_bounds__(kMvThreads) void k_matvec(ProblemView P, int nrhs,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
    __shared__ double sxj[D][kTJ];
    __shared__ double swx[kTJ * kLdw];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const long N = P.N;
    const int r0 = blockIdx.y * 64;
    const long ibase = (long)blockIdx.x * (4 * kRB * 16) + wave * (kRB * 16);
    const int li = lane & 15, lk = lane >> 4;

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
            const long j = j0 + jj;
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
                const double kv = laplace_from_r2<D>(r2);
                a[rb] = (j == irow[rb]) ? 0.0 : kv;
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

template <int D, int NB, int RB>
static void matvec_launch(const ProblemView& P, int nrhs, const double* x, double* y, hipStream_t s) {
    const int rows = 4 * RB * 16;
    dim3 grid((int)((P.N + rows - 1) / rows), (nrhs + 63) / 64);
    hipLaunchKernelGGL((k_matvec<D, NB, RB>), grid, dim3(kMvThreads), 0, s, P, nrhs, x, y);
}

// Row blocks per wave: 4 while the accumulators (RB * NB * 4 doubles) leave room
// for two waves per SIMD, else 2.
template <int D>
static void matvec_d(const ProblemView& P, int nrhs, const double* x, double* y, hipStream_t s) {
    const int groups = (nrhs + 63) / 64;
    const int nb = groups > 1 ? 4 : (nrhs + 15) / 16;
    switch (nb) {
        case 1: matvec_launch<D, 1, 4>(P, nrhs, x, y, s); break;
        case 2: matvec_launch<D, 2, 4>(P, nrhs, x, y, s); break;
        case 3: matvec_launch<D, 3, 2>(P, nrhs, x, y, s); break;
        default: matvec_launch<D, 4, 2>(P, nrhs, x, y, s); break;
    }
}

void launch_matvec(const ProblemView& P, int nrhs, const double* x, double* y, hipStream_t s) {
    if (P.d == 2)
        matvec_d<2>(P, nrhs, x, y, s);
    else
        matvec_d<3>(P, nrhs, x, y, s);
}

}  // namespace cbd
