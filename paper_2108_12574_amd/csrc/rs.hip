// Recursive-skeletonization kernels (Section 3.2): proxy/near-field matrices,
// truncated column-pivoted QR (the ID), box-matrix assembly (e:schur),
// compress-then-eliminate ((e:al), (e:alu), (e:b)), and the level sweeps of
// the factor apply.  Every kernel processes a whole level batch: one
// workgroup per box, all boxes of all subdomains in one launch.
#include <climits>

#include "internal.h"

namespace cbd {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
    for (int o = 32; o > 0; o >>= 1) {
        int u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

// ---- proxy / near-field matrix ---------------------------------------------
// Y_b (m x np, column-major): rows 0..nnear-1 are A(near, p); rows nnear.. are
// K(pxy_q - x_p) w_p for proxy points pxy_q = ctr + rho * dir_q.
template <int D, typename R>
__global__ __launch_bounds__(kThreads) void k_proxy_matrix(ProblemView P,
                                                           const BoxMeta* __restrict__ meta,
                                                           const int* __restrict__ act,
                                                           const int* __restrict__ nearl,
                                                           const int* __restrict__ cidx,
                                                           const double* __restrict__ pxdir,
                                                           int npxy, R* __restrict__ Y) {
    const BoxMeta M = meta[blockIdx.x];
    const long total = (long)M.m * M.np;
    R* Yb = Y + M.y;
    for (long e = (long)blockIdx.y * kThreads + threadIdx.x; e < total; e += (long)gridDim.y * kThreads) {
        const int row = (int)(e % M.m);
        const int col = (int)(e / M.m);
        const long gj = cidx[act[M.act + col]];
        double val;
        if (row < M.nnear) {
            const long gi = cidx[nearl[M.near + row]];
            val = matrix_entry<D>(P, gi, gj);
        } else {
            const int q = row - M.nnear;
            double r2 = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                double dx = M.ctr[t] + M.rho * pxdir[q * D + t] - P.pts[t * P.N + gj];
                r2 += dx * dx;
            }
            val = laplace_from_r2<D>(r2) * P.w[gj];
        }
        Yb[e] = (R)val;
    }
}

template <typename R>
void launch_proxy_matrix(const ProblemView& P, int nbox, const BoxMeta* meta, const int* act,
                         const int* nearl, const int* cidx, const double* pxdir, int npxy, R* Y,
                         hipStream_t s) {
    if (nbox == 0) return;
    dim3 grid(nbox, 8);
    if (P.d == 2)
        hipLaunchKernelGGL((k_proxy_matrix<2, R>), grid, dim3(kThreads), 0, s, P, meta, act, nearl,
                           cidx, pxdir, npxy, Y);
    else
        hipLaunchKernelGGL((k_proxy_matrix<3, R>), grid, dim3(kThreads), 0, s, P, meta, act, nearl,
                           cidx, pxdir, npxy, Y);
}

// ---- truncated CPQR and T = R11^{-1} R12 -----------------------------------
// Businger-Golub pivoting with norms recomputed from the trailing block at every
// step; stop when the largest remaining norm is <= tol * (largest norm of Y).
// Ties: the lowest column position whose norm is within tie * nu0 of the max.
// Writes k, the pivot order (perm: positions, sr: slot ids, skeletons first),
// and T (k x nr, column-major) at the start of the box's factor slot.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_cpqr(const BoxMeta* __restrict__ meta,
                                                   R* __restrict__ Y, const int* __restrict__ act,
                                                   int* __restrict__ sr, int* __restrict__ perm,
                                                   int* __restrict__ kout, R* __restrict__ F,
                                                   R tol, R tie) {
    extern __shared__ char smem_raw[];
    __shared__ R red[kWaves];
    __shared__ int redi[kWaves];
    __shared__ R s_nu0, s_thr;
    __shared__ int s_stop, s_piv, s_k;

    const BoxMeta M = meta[blockIdx.x];
    const int m = M.m, np = M.np;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    R* Yb = Y + M.y;
    R* norms = reinterpret_cast<R*>(smem_raw);   // np
    R* v = norms + np;                           // m
    int* pv = reinterpret_cast<int*>(v + m);     // np

    for (int c = tid; c < np; c += kThreads) pv[c] = c;
    if (tid == 0) s_k = 0;
    __syncthreads();

    const int kmax = m < np ? m : np;
    for (int j = 0; j < kmax; ++j) {
        // remaining column norms
        for (int c = j + wid; c < np; c += kWaves) {
            R s = 0;
            const R* col = Yb + (long)c * m;
            for (int r = j + lane; r < m; r += 64) s += col[r] * col[r];
            s = wave_sum(s);
            if (lane == 0) norms[c] = sqrt(s);
        }
        __syncthreads();
        R lmax = 0;
        for (int c = j + tid; c < np; c += kThreads) lmax = norms[c] > lmax ? norms[c] : lmax;
        lmax = wave_max(lmax);
        if (lane == 0) red[wid] = lmax;
        __syncthreads();
        if (tid == 0) {
            R mx = red[0];
            for (int w = 1; w < kWaves; ++w) mx = red[w] > mx ? red[w] : mx;
            if (j == 0) s_nu0 = mx;
            const R nu0 = s_nu0;
            s_stop = (nu0 == (R)0) || (mx <= tol * nu0);
            s_thr = mx - tie * nu0;
        }
        __syncthreads();
        if (s_stop) break;
        int lmin = INT_MAX;
        for (int c = j + tid; c < np; c += kThreads)
            if (norms[c] >= s_thr) { lmin = c; break; }
        lmin = wave_min_int(lmin);
        if (lane == 0) redi[wid] = lmin;
        __syncthreads();
        if (tid == 0) {
            int p = redi[0];
            for (int w = 1; w < kWaves; ++w) p = redi[w] < p ? redi[w] : p;
            s_piv = p;
        }
        __syncthreads();
        const int piv = s_piv;
        const R xn = norms[piv];
        if (piv != j) {
            R* cj = Yb + (long)j * m;
            R* cp = Yb + (long)piv * m;
            for (int r = tid; r < m; r += kThreads) {
                R t = cj[r];
                cj[r] = cp[r];
                cp[r] = t;
            }
            if (tid == 0) {
                int t = pv[j];
                pv[j] = pv[piv];
                pv[piv] = t;
            }
        }
        __syncthreads();
        const R x0 = Yb[j + (long)j * m];
        const R alpha = x0 >= (R)0 ? -xn : xn;
        const R ax0 = x0 >= (R)0 ? x0 : -x0;
        const R vn2 = (R)2 * xn * xn + (R)2 * ax0 * xn;   // ||x - alpha e1||^2
        for (int r = j + tid; r < m; r += kThreads) v[r - j] = (r == j) ? x0 - alpha : Yb[r + (long)j * m];
        __syncthreads();
        const R beta = vn2 > (R)0 ? (R)2 / vn2 : (R)0;
        for (int c = j + 1 + wid; c < np; c += kWaves) {
            R* col = Yb + (long)c * m;
            R s = 0;
            for (int r = j + lane; r < m; r += 64) s += v[r - j] * col[r];
            s = wave_sum(s) * beta;
            for (int r = j + lane; r < m; r += 64) col[r] -= s * v[r - j];
        }
        if (tid == 0) {
            Yb[j + (long)j * m] = alpha;
            s_k = j + 1;
        }
        __syncthreads();
    }
    __syncthreads();
    const int k = s_k;
    const int nr = np - k;
    if (tid == 0) kout[blockIdx.x] = k;
    for (int c = tid; c < np; c += kThreads) {
        perm[M.act + c] = pv[c];
        sr[M.act + c] = act[M.act + pv[c]];
    }
    // T = R11^{-1} R12 by back substitution, one column per thread
    R* T = F + M.f;
    for (int c = tid; c < nr; c += kThreads) {
        const R* rc = Yb + (long)(k + c) * m;
        for (int a = k - 1; a >= 0; --a) {
            R s = rc[a];
            for (int b = a + 1; b < k; ++b) s -= Yb[a + (long)b * m] * T[b + (long)c * k];
            T[a + (long)c * k] = s / Yb[a + (long)a * m];
        }
    }
}

template <typename R>
void launch_cpqr(int nbox, const BoxMeta* meta, R* Y, const int* act, int* sr, int* perm, int* k,
                 R* F, double tol, double tie, int m_max, int np_max, hipStream_t s) {
    if (nbox == 0) return;
    size_t shm = (size_t)(np_max + m_max) * sizeof(R) + (size_t)np_max * sizeof(int);
    hipLaunchKernelGGL((k_cpqr<R>), dim3(nbox), dim3(kThreads), shm, s, meta, Y, act, sr, perm, k, F,
                       (R)tol, (R)tie);
}

// ---- box matrix A_pp --------------------------------------------------------
// Boxes made of grid points take kernel entries; a parent box takes its
// children's B_ss on the diagonal blocks and kernel entries between children.
template <int D, typename R>
__global__ __launch_bounds__(kThreads) void k_box_matrix(ProblemView P,
                                                         const BoxMeta* __restrict__ meta,
                                                         const int* __restrict__ act,
                                                         const int* __restrict__ cidx,
                                                         const ChildRef<R>* __restrict__ ch,
                                                         R* __restrict__ App) {
    const BoxMeta M = meta[blockIdx.x];
    const int np = M.np;
    const long total = (long)np * np;
    R* A = App + M.app;
    for (long e = (long)blockIdx.y * kThreads + threadIdx.x; e < total; e += (long)gridDim.y * kThreads) {
        const int a = (int)(e % np);
        const int c = (int)(e / np);
        R val;
        if (M.ch >= 0) {
            const ChildRef<R> ra = ch[M.ch + a];
            const ChildRef<R> rc = ch[M.ch + c];
            if (ra.bss == rc.bss) {
                val = ra.bss[ra.pos + (long)rc.pos * ra.ldk];
            } else {
                val = (R)matrix_entry<D>(P, cidx[act[M.act + a]], cidx[act[M.act + c]]);
            }
        } else {
            val = (R)matrix_entry<D>(P, cidx[act[M.act + a]], cidx[act[M.act + c]]);
        }
        A[e] = val;
    }
}

template <typename R>
void launch_box_matrix(const ProblemView& P, int nbox, const BoxMeta* meta, const int* act,
                       const int* cidx, const ChildRef<R>* ch, R* App, hipStream_t s) {
    if (nbox == 0) return;
    dim3 grid(nbox, 16);
    if (P.d == 2)
        hipLaunchKernelGGL((k_box_matrix<2, R>), grid, dim3(kThreads), 0, s, P, meta, act, cidx, ch,
                           App);
    else
        hipLaunchKernelGGL((k_box_matrix<3, R>), grid, dim3(kThreads), 0, s, P, meta, act, cidx, ch,
                           App);
}

// ---- compress-then-eliminate -------------------------------------------------
// With the box matrix permuted to (s, r) order:
//   B_sr = A_sr - A_ss T,  B_rr = A_rr - T^T A_sr - B_sr^T T   ((e:al))
//   B_rr = G^T G,  E = B_sr G^{-1},  B_ss = A_ss - E E^T      ((e:alu), (e:b))
// The factor slot (np x np elements) receives [T | E | G^{-1} | B_ss].
// A root box has k = 0: its slot receives G^{-1} of the whole box matrix.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_eliminate(const BoxMeta* __restrict__ meta,
                                                        const int* __restrict__ perm,
                                                        const int* __restrict__ kk,
                                                        const R* __restrict__ App,
                                                        const double* __restrict__ T64,
                                                        R* __restrict__ Wk, R* __restrict__ F,
                                                        int* __restrict__ status) {
    __shared__ int s_fail;
    const BoxMeta M = meta[blockIdx.x];
    const int np = M.np;
    const int k = kk[blockIdx.x];
    const int nr = np - k;
    const int tid = threadIdx.x;
    const int* pv = perm + M.act;
    const R* A = App + M.app;
    R* Ass = Wk + M.y;
    R* Bsr = Ass + (long)k * k;
    R* Brr = Bsr + (long)k * nr;
    R* Fb = F + M.f;
    R* T = Fb;
    R* E = Fb + (long)k * nr;
    R* Gi = E + (long)k * nr;
    R* Bss = Gi + (long)nr * nr;

    for (long e = tid; e < (long)k * k; e += kThreads) {
        const int a = (int)(e % k), c = (int)(e / k);
        Ass[e] = A[pv[a] + (long)pv[c] * np];
    }
    for (long e = tid; e < (long)k * nr; e += kThreads) {
        const int a = (int)(e % k), i = (int)(e / k);
        Bsr[e] = A[pv[a] + (long)pv[k + i] * np];
    }
    for (long e = tid; e < (long)nr * nr; e += kThreads) {
        const int i = (int)(e % nr), c = (int)(e / nr);
        Brr[e] = A[pv[k + i] + (long)pv[k + c] * np];
    }
    // T of the ID (computed in FP64) in the factor's precision
    for (long e = tid; e < (long)k * nr; e += kThreads) T[e] = (R)T64[M.f + e];
    if (tid == 0) s_fail = 0;
    __syncthreads();

    if (k > 0 && nr > 0) {
        // B_rr -= T^T A_sr   (Bsr still holds A_sr)
        for (long e = tid; e < (long)nr * nr; e += kThreads) {
            const int i = (int)(e % nr), c = (int)(e / nr);
            R s = 0;
            for (int a = 0; a < k; ++a) s += T[a + (long)i * k] * Bsr[a + (long)c * k];
            Brr[e] -= s;
        }
        __syncthreads();
        // B_sr = A_sr - A_ss T  (in place: each entry reads only its own A_sr value)
        for (long e = tid; e < (long)k * nr; e += kThreads) {
            const int a = (int)(e % k), i = (int)(e / k);
            R s = 0;
            for (int b = 0; b < k; ++b) s += Ass[a + (long)b * k] * T[b + (long)i * k];
            Bsr[e] -= s;
        }
        __syncthreads();
        // B_rr -= B_sr^T T
        for (long e = tid; e < (long)nr * nr; e += kThreads) {
            const int i = (int)(e % nr), c = (int)(e / nr);
            R s = 0;
            for (int a = 0; a < k; ++a) s += Bsr[a + (long)i * k] * T[a + (long)c * k];
            Brr[e] -= s;
        }
        __syncthreads();
    }
    // symmetrize the upper triangle
    for (long e = tid; e < (long)nr * nr; e += kThreads) {
        const int i = (int)(e % nr), c = (int)(e / nr);
        if (i < c) Brr[e] = (R)0.5 * (Brr[e] + Brr[c + (long)i * nr]);
    }
    __syncthreads();
    // right-looking Cholesky, upper triangle in place: B_rr = G^T G
    for (int j = 0; j < nr; ++j) {
        if (tid == 0) {
            const R dj = Brr[j + (long)j * nr];
            if (!(dj > (R)0)) s_fail = 1;
            else Brr[j + (long)j * nr] = sqrt(dj);
        }
        __syncthreads();
        if (s_fail) break;
        const R g = Brr[j + (long)j * nr];
        for (int c = j + 1 + tid; c < nr; c += kThreads) Brr[j + (long)c * nr] /= g;
        __syncthreads();
        const int rem = nr - j - 1;
        for (long e = tid; e < (long)rem * rem; e += kThreads) {
            const int a = j + 1 + (int)(e % rem), c = j + 1 + (int)(e / rem);
            if (a <= c) Brr[a + (long)c * nr] -= Brr[j + (long)a * nr] * Brr[j + (long)c * nr];
        }
        __syncthreads();
    }
    if (s_fail) {
        if (tid == 0) status[0] = blockIdx.x + 1;
        return;
    }
    // G^{-1} (upper): column c solves G x = e_c by back substitution
    for (int c = tid; c < nr; c += kThreads) {
        for (int a = nr - 1; a > c; --a) Gi[a + (long)c * nr] = (R)0;
        Gi[c + (long)c * nr] = (R)1 / Brr[c + (long)c * nr];
        for (int a = c - 1; a >= 0; --a) {
            R s = 0;
            for (int b = a + 1; b <= c; ++b) s += Brr[a + (long)b * nr] * Gi[b + (long)c * nr];
            Gi[a + (long)c * nr] = -s / Brr[a + (long)a * nr];
        }
    }
    __syncthreads();
    // E = B_sr G^{-1}
    for (long e = tid; e < (long)k * nr; e += kThreads) {
        const int a = (int)(e % k), i = (int)(e / k);
        R s = 0;
        for (int j = 0; j <= i; ++j) s += Bsr[a + (long)j * k] * Gi[j + (long)i * nr];
        E[e] = s;
    }
    __syncthreads();
    // B_ss = A_ss - E E^T
    for (long e = tid; e < (long)k * k; e += kThreads) {
        const int a = (int)(e % k), c = (int)(e / k);
        R s = 0;
        for (int i = 0; i < nr; ++i) s += E[a + (long)i * k] * E[c + (long)i * k];
        Bss[e] = Ass[e] - s;
    }
}

template <typename R>
void launch_eliminate(int nbox, const BoxMeta* meta, const int* perm, const int* k, const R* App,
                      const double* T64, R* Wk, R* F, int* status, hipStream_t s) {
    if (nbox == 0) return;
    hipLaunchKernelGGL((k_eliminate<R>), dim3(nbox), dim3(kThreads), 0, s, meta, perm, k, App, T64, Wk,
                       F, status);
}

// ---- apply ------------------------------------------------------------------
// v: local vectors of all subdomains, slot-major (v[slot * nrhs + c]).
template <typename R>
__global__ void k_gather(const double* __restrict__ r, long N, int nrhs, const int* __restrict__ cidx,
                         long total, R* __restrict__ v) {
    const long n = total * nrhs;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long slot = e / nrhs;
        const int c = (int)(e % nrhs);
        v[e] = (R)r[(long)c * N + cidx[slot]];
    }
}

template <typename R>
void launch_gather(const double* r, long N, int nrhs, const int* cidx, long total, R* v,
                   hipStream_t s) {
    long n = total * nrhs;
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL((k_gather<R>), dim3((int)b), dim3(256), 0, s, r, N, nrhs, cidx, total, v);
}

// z[:, g] = sum over the subdomain slots holding point g, in a fixed order
template <typename R>
__global__ void k_scatter(const R* __restrict__ v, int nrhs, const int* __restrict__ inv_ptr,
                          const int* __restrict__ inv_slot, long N, double* __restrict__ z) {
    const long n = N * nrhs;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
        const long g = e % N;
        const int c = (int)(e / N);
        double s = 0.0;
        for (int q = inv_ptr[g]; q < inv_ptr[g + 1]; ++q) s += (double)v[(long)inv_slot[q] * nrhs + c];
        z[e] = s;
    }
}

template <typename R>
void launch_scatter(const R* v, int nrhs, const int* inv_ptr, const int* inv_slot, long N, double* z,
                    hipStream_t s) {
    long n = N * nrhs;
    long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    hipLaunchKernelGGL((k_scatter<R>), dim3((int)b), dim3(256), 0, s, v, nrhs, inv_ptr, inv_slot, N, z);
}

// One level of the apply sweep, one workgroup per (box, chunk of rc columns).
// forward:  t = v_r - T^T v_s;  v_r = G^{-T} t;  v_s -= E v_r
// backward: t = v_r - E^T v_s;  v_r = G^{-1} t;  v_s -= T v_r
template <typename R>
__global__ __launch_bounds__(kThreads) void k_apply_level(const BoxMeta* __restrict__ meta,
                                                          const int* __restrict__ sr,
                                                          const int* __restrict__ kk,
                                                          const R* __restrict__ F, R* __restrict__ v,
                                                          int nrhs, int rc, int forward) {
    extern __shared__ char smem_raw[];
    const BoxMeta M = meta[blockIdx.x];
    const int np = M.np, k = kk[blockIdx.x], nr = np - k;
    const int c0 = blockIdx.y * rc;
    const int nc = (nrhs - c0) < rc ? (nrhs - c0) : rc;
    const int tid = threadIdx.x;
    R* sv = reinterpret_cast<R*>(smem_raw);   // np x rc, rows s then r
    R* tmp = sv + (long)np * rc;              // nr x rc
    const int* ix = sr + M.act;
    for (long e = tid; e < (long)np * nc; e += kThreads) {
        const int a = (int)(e / nc), c = (int)(e % nc);
        sv[a * rc + c] = v[(long)ix[a] * nrhs + c0 + c];
    }
    __syncthreads();
    if (nr > 0) {
        const R* T = F + M.f;
        const R* E = T + (long)k * nr;
        const R* Gi = E + (long)k * nr;
        R* vs = sv;
        R* vr = sv + (long)k * rc;
        const R* X1 = forward ? T : E;   // applied first (transposed)
        const R* X2 = forward ? E : T;   // applied last
        for (long e = tid; e < (long)nr * nc; e += kThreads) {
            const int i = (int)(e / nc), c = (int)(e % nc);
            R s = vr[i * rc + c];
            for (int a = 0; a < k; ++a) s -= X1[a + (long)i * k] * vs[a * rc + c];
            tmp[i * rc + c] = s;
        }
        __syncthreads();
        for (long e = tid; e < (long)nr * nc; e += kThreads) {
            const int i = (int)(e / nc), c = (int)(e % nc);
            R s = 0;
            if (forward) {
                for (int j = 0; j <= i; ++j) s += Gi[j + (long)i * nr] * tmp[j * rc + c];
            } else {
                for (int j = i; j < nr; ++j) s += Gi[i + (long)j * nr] * tmp[j * rc + c];
            }
            vr[i * rc + c] = s;
        }
        __syncthreads();
        for (long e = tid; e < (long)k * nc; e += kThreads) {
            const int a = (int)(e / nc), c = (int)(e % nc);
            R s = vs[a * rc + c];
            for (int i = 0; i < nr; ++i) s -= X2[a + (long)i * k] * vr[i * rc + c];
            vs[a * rc + c] = s;
        }
        __syncthreads();
    }
    for (long e = tid; e < (long)np * nc; e += kThreads) {
        const int a = (int)(e / nc), c = (int)(e % nc);
        v[(long)ix[a] * nrhs + c0 + c] = sv[a * rc + c];
    }
}

template <typename R>
void launch_apply_level(int nbox, const BoxMeta* meta, const int* sr, const int* k, const R* F, R* v,
                        int nrhs, int np_max, bool forward, hipStream_t s) {
    if (nbox == 0) return;
    // columns per workgroup so that the local copy fits in 64 KiB of LDS
    int rc = 16;
    while (rc > 1 && (size_t)2 * np_max * rc * sizeof(R) > 65536) rc >>= 1;
    if (rc > nrhs) rc = nrhs;
    size_t shm = (size_t)2 * np_max * rc * sizeof(R);
    dim3 grid(nbox, (nrhs + rc - 1) / rc);
    hipLaunchKernelGGL((k_apply_level<R>), grid, dim3(kThreads), shm, s, meta, sr, k, F, v, nrhs, rc,
                       forward ? 1 : 0);
}

// explicit instantiations
template void launch_proxy_matrix<double>(const ProblemView&, int, const BoxMeta*, const int*,
                                          const int*, const int*, const double*, int, double*,
                                          hipStream_t);
template void launch_cpqr<double>(int, const BoxMeta*, double*, const int*, int*, int*, int*, double*,
                                  double, double, int, int, hipStream_t);
#define CBD_INST(R)                                                                                 \
    template void launch_box_matrix<R>(const ProblemView&, int, const BoxMeta*, const int*,         \
                                       const int*, const ChildRef<R>*, R*, hipStream_t);            \
    template void launch_eliminate<R>(int, const BoxMeta*, const int*, const int*, const R*,       \
                                      const double*, R*, R*, int*, hipStream_t);                    \
    template void launch_gather<R>(const double*, long, int, const int*, long, R*, hipStream_t);   \
    template void launch_scatter<R>(const R*, int, const int*, const int*, long, double*,          \
                                    hipStream_t);                                                   \
    template void launch_apply_level<R>(int, const BoxMeta*, const int*, const int*, const R*, R*,  \
                                        int, int, bool, hipStream_t);
CBD_INST(double)
CBD_INST(float)
#undef CBD_INST

}  // namespace cbd
