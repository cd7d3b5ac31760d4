// Matvec by FFT on the uniform grid (the paper's choice, Section 5): the kernel
// part of A x is the aperiodic convolution of u = w o x with g[delta] =
// K(spacing * |delta|) (g[0] = 0; the diagonal is added separately), computed by
// circulant embedding in a P^d grid, P = a power of two >= 2n - 1.  g is even,
// so its transform is real and two real right-hand sides travel in one complex
// transform (real and imaginary parts stay separate).  The transforms are
// radix-2 line FFTs in LDS, one workgroup per line, batched over lines and
// right-hand-side pairs.
#include "internal.h"

namespace cbd {

constexpr int kFftThreads = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place transform of the lines of axis `axis` of `batch` P^d arrays (x fastest):
// line l of array q starts at q*P^d + (l % inner) + (l / inner) * inner * P, with
// element stride inner = P^axis.  tw[k] = exp(-2 pi i k / P), k < P/2.
__global__ __launch_bounds__(kFftThreads) void k_fft_lines(double2* __restrict__ data, int P, int logP,
                                                           long vol, long inner, const double2* __restrict__ tw,
                                                           int inverse) {
    extern __shared__ double2 s[];
    const long line = blockIdx.x;
    const long base = (long)blockIdx.y * vol + (line % inner) + (line / inner) * inner * P;
    for (int t = threadIdx.x; t < P; t += kFftThreads) {
        const int r = (int)(__brev((unsigned)t) >> (32 - logP));
        s[r] = data[base + (long)t * inner];
    }
    __syncthreads();
    for (int len = 2; len <= P; len <<= 1) {
        const int half = len >> 1, step = P / len;
        for (int b = threadIdx.x; b < P / 2; b += kFftThreads) {
            const int pos = b % half;
            const int i = (b / half) * len + pos, j = i + half;
            double2 w = tw[pos * step];
            if (inverse) w.y = -w.y;
            const double2 u = s[i], v = cmul(s[j], w);
            s[i] = make_double2(u.x + v.x, u.y + v.y);
            s[j] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    const double sc = inverse ? 1.0 / P : 1.0;
    for (int t = threadIdx.x; t < P; t += kFftThreads)
        data[base + (long)t * inner] = make_double2(s[t].x * sc, s[t].y * sc);
}

// Circulant generator of the kernel: g at every P^d index (real part), g[0] = 0.
template <int D>
__global__ void k_fft_generator(double2* __restrict__ g, int n, int P, double spacing) {
    long vol = 1;
    for (int t = 0; t < D; ++t) vol *= P;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < vol; e += (long)gridDim.x * blockDim.x) {
        long rem = e;
        double r2 = 0.0;
        bool in = true;
        for (int t = 0; t < D; ++t) {
            const int i = (int)(rem % P);
            rem /= P;
            int dlt = i < n ? i : i - P;            // |delta| < n, else outside the embedding
            if (i >= n && i <= P - n) in = false;
            const double dx = spacing * dlt;
            r2 += dx * dx;
        }
        g[e] = make_double2(in && r2 > 0.0 ? laplace_from_r2<D>(r2) : 0.0, 0.0);
    }
}

// Pack right-hand sides 2q, 2q+1 (of the chunk starting at c0) as u = w x into pair q.
template <int D>
__global__ void k_fft_pack(const ProblemView Pv, int P, int nrhs, int c0, int pairs, const double* __restrict__ x,
                           double2* __restrict__ buf) {
    long vol = 1;
    for (int t = 0; t < D; ++t) vol *= P;
    const long total = vol * pairs;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int q = (int)(e / vol);
        long rem = e % vol, g = 0, mul = 1;
        bool in = true;
        for (int t = 0; t < D; ++t) {
            const int i = (int)(rem % P);
            rem /= P;
            if (i >= Pv.n) in = false;
            g += i * mul;
            mul *= Pv.n;
        }
        double2 v = make_double2(0.0, 0.0);
        if (in) {
            const int ca = c0 + 2 * q, cb = ca + 1;
            const double w = Pv.w[g];
            v.x = w * x[(long)ca * Pv.N + g];
            if (cb < nrhs) v.y = w * x[(long)cb * Pv.N + g];
        }
        buf[e] = v;
    }
}

__global__ void k_fft_scale(double2* __restrict__ buf, const double* __restrict__ ghat, long vol, int pairs) {
    const long total = vol * pairs;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const double s = ghat[e % vol];
        buf[e] = make_double2(buf[e].x * s, buf[e].y * s);
    }
}

template <int D>
__global__ void k_fft_unpack(const ProblemView Pv, int P, int nrhs, int c0, int pairs, const double* __restrict__ x,
                             const double2* __restrict__ buf, double* __restrict__ y) {
    const long total = Pv.N * pairs;
    long vol = 1;
    for (int t = 0; t < D; ++t) vol *= P;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int q = (int)(e / Pv.N);
        const long g = e % Pv.N;
        long rem = g, idx = 0, mul = 1;
        for (int t = 0; t < D; ++t) {
            idx += (rem % Pv.n) * mul;
            rem /= Pv.n;
            mul *= P;
        }
        const double2 v = buf[(long)q * vol + idx];
        const int ca = c0 + 2 * q, cb = ca + 1;
        const double bi = Pv.rs[g], di = Pv.diag[g];
        y[(long)ca * Pv.N + g] = bi * v.x + di * x[(long)ca * Pv.N + g];
        if (cb < nrhs) y[(long)cb * Pv.N + g] = bi * v.y + di * x[(long)cb * Pv.N + g];
    }
}

__global__ void k_fft_real(const double2* __restrict__ a, double* __restrict__ r, long n) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) r[e] = a[e].x;
}

static int grid_for(long n) {
    long b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    return (int)(b < 1 ? 1 : b);
}

static void fft_all_axes(double2* buf, int d, int P, int logP, int batch, const double2* tw, int inverse,
                         hipStream_t s) {
    long vol = 1;
    for (int t = 0; t < d; ++t) vol *= P;
    long inner = 1;
    for (int a = 0; a < d; ++a) {
        CBD_LAUNCH(k_fft_lines, dim3((unsigned)(vol / P), batch), dim3(kFftThreads),
                           (size_t)P * sizeof(double2), s, buf, P, logP, vol, inner, tw, inverse);
        inner *= P;
    }
}

void launch_fft_prepare(const ProblemView& Pv, int P, int logP, double spacing, double2* gbuf, double* ghat,
                        const double2* tw, hipStream_t s) {
    long vol = 1;
    for (int t = 0; t < Pv.d; ++t) vol *= P;
    if (Pv.d == 2)
        CBD_LAUNCH(k_fft_generator<2>, dim3(grid_for(vol)), dim3(256), 0, s, gbuf, Pv.n, P, spacing);
    else
        CBD_LAUNCH(k_fft_generator<3>, dim3(grid_for(vol)), dim3(256), 0, s, gbuf, Pv.n, P, spacing);
    fft_all_axes(gbuf, Pv.d, P, logP, 1, tw, 0, s);
    // the transform of the even generator is real: keep the real part
    CBD_LAUNCH(k_fft_real, dim3(grid_for(vol)), dim3(256), 0, s, gbuf, ghat, vol);
}

void launch_matvec_fft(const ProblemView& Pv, int P, int logP, const double* ghat, const double2* tw,
                       double2* buf, int max_pairs, int nrhs, const double* x, double* y, hipStream_t s) {
    long vol = 1;
    for (int t = 0; t < Pv.d; ++t) vol *= P;
    for (int c0 = 0; c0 < nrhs; c0 += 2 * max_pairs) {
        const int pairs = (int)((nrhs - c0 + 1) / 2 < max_pairs ? (nrhs - c0 + 1) / 2 : max_pairs);
        if (Pv.d == 2)
            CBD_LAUNCH(k_fft_pack<2>, dim3(grid_for(vol * pairs)), dim3(256), 0, s, Pv, P, nrhs, c0, pairs,
                               x, buf);
        else
            CBD_LAUNCH(k_fft_pack<3>, dim3(grid_for(vol * pairs)), dim3(256), 0, s, Pv, P, nrhs, c0, pairs,
                               x, buf);
        fft_all_axes(buf, Pv.d, P, logP, pairs, tw, 0, s);
        CBD_LAUNCH(k_fft_scale, dim3(grid_for(vol * pairs)), dim3(256), 0, s, buf, ghat, vol, pairs);
        fft_all_axes(buf, Pv.d, P, logP, pairs, tw, 1, s);
        if (Pv.d == 2)
            CBD_LAUNCH(k_fft_unpack<2>, dim3(grid_for(Pv.N * pairs)), dim3(256), 0, s, Pv, P, nrhs, c0,
                               pairs, x, buf, y);
        else
            CBD_LAUNCH(k_fft_unpack<3>, dim3(grid_for(Pv.N * pairs)), dim3(256), 0, s, Pv, P, nrhs, c0,
                               pairs, x, buf, y);
    }
}

}  // namespace cbd
