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

// y[:, r0:r0+RC] = A x[:, r0:r0+RC].  One thread per row i; the columns j are
// streamed through LDS in tiles of 256 points (coordinates and w_j x_j), and
// every kernel value K(x_i - x_j) is evaluated once for the RC right-hand sides.
constexpr int kMvThreads = 256;

template <int D, int RC>
__global__ __launch_bounds__(kMvThreads) void k_matvec(ProblemView P, int nrhs,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
    __shared__ double sp[D][kMvThreads];
    __shared__ double swx[RC][kMvThreads];
    const int tid = threadIdx.x;
    const long N = P.N;
    const long i = (long)blockIdx.x * kMvThreads + tid;
    const int r0 = blockIdx.y * RC;
    double xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = (i < N) ? P.pts[t * N + i] : 0.0;
    double acc[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) acc[r] = 0.0;

    for (long j0 = 0; j0 < N; j0 += kMvThreads) {
        __syncthreads();
        long j = j0 + tid;
        if (j < N) {
#pragma unroll
            for (int t = 0; t < D; ++t) sp[t][tid] = P.pts[t * N + j];
            double wj = P.w[j];
#pragma unroll
            for (int r = 0; r < RC; ++r)
                swx[r][tid] = (r0 + r < nrhs) ? wj * x[(long)(r0 + r) * N + j] : 0.0;
        }
        __syncthreads();
        const int jn = (N - j0 < kMvThreads) ? (int)(N - j0) : kMvThreads;
        for (int jj = 0; jj < jn; ++jj) {
            double r2 = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                double dx = xi[t] - sp[t][jj];
                r2 += dx * dx;
            }
            double kv = (j0 + jj == i) ? 0.0 : laplace_from_r2<D>(r2);
#pragma unroll
            for (int r = 0; r < RC; ++r) acc[r] += kv * swx[r][jj];
        }
    }
    if (i < N) {
        const double bi = P.rs[i], di = P.diag[i];
#pragma unroll
        for (int r = 0; r < RC; ++r)
            if (r0 + r < nrhs) y[(long)(r0 + r) * N + i] = bi * acc[r] + di * x[(long)(r0 + r) * N + i];
    }
}

template <int D>
static void matvec_d(const ProblemView& P, int nrhs, const double* x, double* y, hipStream_t s) {
    int blocks = (int)((P.N + kMvThreads - 1) / kMvThreads);
    if (nrhs == 1) {
        hipLaunchKernelGGL((k_matvec<D, 1>), dim3(blocks, 1), dim3(kMvThreads), 0, s, P, nrhs, x, y);
    } else if (nrhs <= 4) {
        hipLaunchKernelGGL((k_matvec<D, 4>), dim3(blocks, 1), dim3(kMvThreads), 0, s, P, nrhs, x, y);
    } else if (nrhs <= 8) {
        hipLaunchKernelGGL((k_matvec<D, 8>), dim3(blocks, 1), dim3(kMvThreads), 0, s, P, nrhs, x, y);
    } else {
        int chunks = (nrhs + 15) / 16;
        hipLaunchKernelGGL((k_matvec<D, 16>), dim3(blocks, chunks), dim3(kMvThreads), 0, s, P, nrhs,
                           x, y);
    }
}

void launch_matvec(const ProblemView& P, int nrhs, const double* x, double* y, hipStream_t s) {
    if (P.d == 2)
        matvec_d<2>(P, nrhs, x, y, s);
    else
        matvec_d<3>(P, nrhs, x, y, s);
}

}  // namespace cbd
