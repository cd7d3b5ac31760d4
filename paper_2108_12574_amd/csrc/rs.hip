// Recursive-skeletonization kernels (Section 4.2): proxy/near-field matrices,
// truncated column-pivoted QR (the ID), box-matrix assembly (e:schur),
// compress-then-eliminate ((e:al), (e:alu), (e:b)), and the level sweeps of
// the factor apply.  Every kernel processes a whole level batch: one
// workgroup per box, all boxes of all subdomains in one launch.
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

namespace cbd {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Wave-wide reductions by DPP lane moves (no LDS round trips): quad_perm [1,0,3,2] and
// [2,3,0,1] combine lanes l ^ 1 and l ^ 2, row_ror 4 and 8 the four quads of each row
// of 16 lanes, and the four row results are read from lanes 0, 16, 32 and 48.  Every
// lane returns the total.  A double moves as its two 32-bit halves.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRor4 = 0x124, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppRor4>(v);
    v += dpp_f64<kDppRor8>(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppRor4>(v));
    v = fmax(v, dpp_f64<kDppRor8>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}
__device__ __forceinline__ int wave_min_int(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppXor1, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppXor2, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppRor4, 0xF, 0xF, true));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, kDppRor8, 0xF, 0xF, true));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Largest dynamic LDS `kernel` may take on the current device: the device's LDS per
// workgroup less 1 KB for the kernel's own arrays (160 KB per workgroup on gfx950).
// Above 64 KB a launch needs the kernel's attribute raised, which is done here once
// per kernel and device (64 KB less 1 KB if that fails).
size_t dyn_lds_limit(const void* kernel) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> lim;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 65536 - 1024;
    std::lock_guard<std::mutex> lock(mu);
    size_t& l = lim[{kernel, dev}];
    if (!l) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        l = (size_t)v - 1024;
        if (l > 65536 && hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)l) != hipSuccess)
            l = 65536 - 1024;
    }
    return l;
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
    // rows (near-field points, then proxy points) staged in LDS in chunks of kPxRows:
    // coordinates, row scale (1 for proxy rows) and grid index (-1 for proxy rows);
    // the workgroup's columns then run over the chunk with one row per thread
    constexpr int kPxRows = 512;
    __shared__ double sx[D][kPxRows];
    __shared__ double srs[kPxRows];
    __shared__ long sgi[kPxRows];
    const BoxMeta M = meta[blockIdx.x];
    const int per = (M.np + gridDim.y - 1) / gridDim.y;
    const int c_lo = blockIdx.y * per, c_hi = min(M.np, c_lo + per);
    if (c_lo >= c_hi) return;
    const int tid = threadIdx.x;
    R* Yb = Y + M.y;
    for (int r0 = 0; r0 < M.m; r0 += kPxRows) {
        const int nrow = min(kPxRows, M.m - r0);
        __syncthreads();
        for (int rr = tid; rr < nrow; rr += kThreads) {
            const int row = r0 + rr;
            if (row < M.nnear) {
                const long gi = cidx[nearl[M.near + row]];
#pragma unroll
                for (int t = 0; t < D; ++t) sx[t][rr] = P.pts[t * P.N + gi];
                srs[rr] = P.rs[gi];
                sgi[rr] = gi;
            } else {
                const int q = row - M.nnear;
#pragma unroll
                for (int t = 0; t < D; ++t) sx[t][rr] = M.ctr[t] + M.rho * pxdir[q * D + t];
                srs[rr] = 1.0;
                sgi[rr] = -1;
            }
        }
        __syncthreads();
        for (int col = c_lo; col < c_hi; ++col) {
            const long gj = cidx[act[M.act + col]];
            double xj[D];
#pragma unroll
            for (int t = 0; t < D; ++t) xj[t] = P.pts[t * P.N + gj];
            const double wj = P.w[gj];
            R* yc = Yb + (long)col * M.m + r0;
            for (int rr = tid; rr < nrow; rr += kThreads) {
                double val;
                if (sgi[rr] == gj) {
                    val = P.diag[gj];
                } else {
                    double r2 = 0.0;
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const double dx = sx[t][rr] - xj[t];
                        r2 += dx * dx;
                    }
                    val = srs[rr] * laplace_from_r2<D>(r2) * wj;
                }
                yc[rr] = (R)val;
            }
        }
    }
}

template <typename R>
void launch_proxy_matrix(const ProblemView& P, int nbox, const BoxMeta* meta, const int* act,
                         const int* nearl, const int* cidx, const double* pxdir, int npxy, R* Y,
                         hipStream_t s) {
    if (nbox == 0) return;
    dim3 grid(nbox, 8);
    if (P.d == 2)
        CBD_LAUNCH((k_proxy_matrix<2, R>), grid, dim3(kThreads), 0, s, P, meta, act, nearl,
                           cidx, pxdir, npxy, Y);
    else
        CBD_LAUNCH((k_proxy_matrix<3, R>), grid, dim3(kThreads), 0, s, P, meta, act, nearl,
                           cidx, pxdir, npxy, Y);
}

// ---- truncated CPQR and T = R11^{-1} R12 -----------------------------------
// Businger-Golub pivoting: at every step the column with the largest remaining
// norm (over the rows not yet eliminated) is swapped to the front and reduced by
// a Householder reflection; stop when that norm is <= tol * nu0 (nu0: largest
// column norm of Y).  Ties: the lowest column position whose norm is within
// tie * nu0 of the maximum.  The remaining norms are recomputed from the updated
// trailing block in the same pass as the reflection (no down-dating).
// Outputs: k, the pivot order (perm: positions, sr: slot ids, skeletons first),
// and T (k x nr, column-major) at the box's factor offset of T64.

// Columns [c_lo, c_hi) of T = R11^{-1} R12 (R in the first k rows of Yb, ld m;
// T k x nr with ld k); defined below.  Columns are independent, so the T of a box
// may be split over workgroups.
__device__ void id_coefficients(const double* Yb, int m, int np, int k, double* T, int c_lo, int c_hi);

// Householder update of trailing columns c in [c_lo, c_hi) (c > j) with the
// reflector v (LDS, rows j..m-1), then their norm over rows j+1..m-1.  Wave w
// takes the columns c_lo + w + kWaves t, four at a time, so that the loads of
// four columns are in flight together; each column's arithmetic (and so its
// rounding) does not depend on the grouping.
__device__ __forceinline__ void reflect_columns(double* Yb, int m, int j, int c_lo, int c_hi,
                                                const double* v, double beta, double* norms) {
    constexpr int G = 4;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c0 = c_lo + wid; c0 < c_hi; c0 += G * kWaves) {
        double* col[G];
        bool ok[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int c = c0 + u * kWaves;
            ok[u] = c < c_hi;
            col[u] = Yb + (long)(ok[u] ? c : c0) * m;
        }
        double sd[G];
#pragma unroll
        for (int u = 0; u < G; ++u) sd[u] = 0.0;
        for (int r = j + lane; r < m; r += 64) {
            const double vv = v[r - j];
#pragma unroll
            for (int u = 0; u < G; ++u) sd[u] += vv * col[u][r];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) sd[u] = wave_sum(sd[u]) * beta;
        double q[G];
#pragma unroll
        for (int u = 0; u < G; ++u) q[u] = 0.0;
        for (int r = j + lane; r < m; r += 64) {
            const double vv = v[r - j];
            double y[G];
#pragma unroll
            for (int u = 0; u < G; ++u) y[u] = col[u][r] - sd[u] * vv;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (!ok[u]) continue;
                col[u][r] = y[u];
                if (r > j) q[u] += y[u] * y[u];
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            q[u] = wave_sum(q[u]);
            if (lane == 0 && ok[u]) norms[c0 + u * kWaves] = sqrt(q[u]);
        }
    }
}

// Register-resident form of reflect_columns for m - j <= 64 NR rows: a wave loads
// all rows of G columns at once, so the loads of a column are in flight together
// and the column is read once.  The loads and stores go through a buffer resource
// per column (base in scalar registers, one offset register for all rows; loads
// past the column's end return 0, where the reflector is 0 too).  The per-lane
// sums run over the same rows in the same order as reflect_columns, so the results
// are the same.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const double* Yb, int m, int j, int c, int rows) {
    // 0x00020000: the gfx9 buffer-resource word 3 for raw (untyped) accesses
    return __builtin_amdgcn_make_buffer_rsrc((void*)(Yb + (long)c * m + j), (short)0, rows * (int)sizeof(double),
                                             0x00020000);
}

template <int NR>
__device__ __forceinline__ void reflect_columns_reg(double* Yb, int m, int j, int c_lo, int c_hi,
                                                    const double* v, double beta, double* norms) {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(__amdgpu_buffer_rsrc_t(), 0, 0, 0)) b64;
    constexpr int G = NR > 12 ? 1 : 2;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // column bases in SGPRs
    const int rows = m - j;
    for (int c0 = c_lo + wid; c0 < c_hi; c0 += G * kWaves) {
        __amdgpu_buffer_rsrc_t rs[G];
        bool ok[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int c = c0 + u * kWaves;
            ok[u] = c < c_hi;
            rs[u] = column_rsrc(Yb, m, j, ok[u] ? c : c0, rows);
        }
        double a[G][NR];
#pragma unroll
        for (int i = 0; i < NR; ++i)
#pragma unroll
            for (int u = 0; u < G; ++u)
                a[u][i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs[u], (lane + 64 * i) * 8, 0, 0));
        double sd[G];
#pragma unroll
        for (int u = 0; u < G; ++u) sd[u] = 0.0;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rr = lane + 64 * i;
            const double vv = rr < rows ? v[rr] : 0.0;
#pragma unroll
            for (int u = 0; u < G; ++u) sd[u] += vv * a[u][i];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) sd[u] = wave_sum(sd[u]) * beta;
        // compiler-only barrier: the reflector is read from LDS again below instead of
        // being kept in registers through the reduction
        __asm__ volatile("" ::: "memory");
        double q[G];
#pragma unroll
        for (int u = 0; u < G; ++u) q[u] = 0.0;
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const int rr = lane + 64 * i;
            if (rr < rows) {
                const double vv = v[rr];
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const double y = a[u][i] - sd[u] * vv;
                    if (ok[u]) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64, y), rs[u], rr * 8, 0, 0);
                    if (rr > 0) q[u] += y * y;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            q[u] = wave_sum(q[u]);
            if (lane == 0 && ok[u]) norms[c0 + u * kWaves] = sqrt(q[u]);
        }
    }
}

// One workgroup per box (levels with many boxes).  The column update keeps up to
// 64 NRMAX rows in registers (the instantiation is chosen by the largest box).
template <int NRMAX>
__global__ __launch_bounds__(kThreads) void k_cpqr(const BoxMeta* __restrict__ meta,
                                                   double* __restrict__ Y, const int* __restrict__ act,
                                                   int* __restrict__ sr, int* __restrict__ perm,
                                                   int* __restrict__ kout, double* __restrict__ T64,
                                                   double tol, double tie) {
    extern __shared__ char smem_raw[];
    __shared__ double red[kWaves];
    __shared__ int redi[kWaves];
    __shared__ double s_nu0, s_thr;
    __shared__ int s_stop, s_piv, s_k;

    const BoxMeta M = meta[blockIdx.x];
    const int m = M.m, np = M.np;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double* Yb = Y + M.y;
    double* norms = reinterpret_cast<double*>(smem_raw);   // np
    double* v = norms + np;                                 // m
    int* pv = reinterpret_cast<int*>(v + m);                // np

    for (int c = tid; c < np; c += kThreads) pv[c] = c;
    for (int c = wid; c < np; c += kWaves) {
        const double* col = Yb + (long)c * m;
        double q = 0;
        for (int r = lane; r < m; r += 64) q += col[r] * col[r];
        q = wave_sum(q);
        if (lane == 0) norms[c] = sqrt(q);
    }
    if (tid == 0) s_k = 0;
    __syncthreads();

    const int kmax = m < np ? m : np;
    for (int j = 0; j < kmax; ++j) {
        double lmax = 0;
        for (int c = j + tid; c < np; c += kThreads) lmax = norms[c] > lmax ? norms[c] : lmax;
        lmax = wave_max(lmax);
        if (lane == 0) red[wid] = lmax;
        __syncthreads();
        if (tid == 0) {
            double mx = red[0];
            for (int w = 1; w < kWaves; ++w) mx = red[w] > mx ? red[w] : mx;
            if (j == 0) s_nu0 = mx;
            const double nu0 = s_nu0;
            s_stop = (nu0 == 0.0) || (mx <= tol * nu0);
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
        const double xn = norms[piv];
        if (piv != j) {
            double* cj = Yb + (long)j * m;
            double* cp = Yb + (long)piv * m;
            for (int r = tid; r < m; r += kThreads) {
                const double t = cj[r];
                cj[r] = cp[r];
                cp[r] = t;
            }
        }
        __syncthreads();
        // (column piv now holds the old column j; its norm is recomputed below)
        if (tid == 0 && piv != j) {
            const int t = pv[j];
            pv[j] = pv[piv];
            pv[piv] = t;
        }
        const double x0 = Yb[j + (long)j * m];
        const double alpha = x0 >= 0.0 ? -xn : xn;
        const double vn2 = 2.0 * xn * xn + 2.0 * fabs(x0) * xn;   // ||x - alpha e1||^2
        for (int r = j + tid; r < m; r += kThreads) v[r - j] = (r == j) ? x0 - alpha : Yb[r + (long)j * m];
        __syncthreads();
        const double beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        // (the row count is uniform over the workgroup)
        if (m - j <= 256)
            reflect_columns_reg<4>(Yb, m, j, j + 1, np, v, beta, norms);
        else if (m - j <= 512)
            reflect_columns_reg<8>(Yb, m, j, j + 1, np, v, beta, norms);
        else if (NRMAX >= 12 && m - j <= 768)
            reflect_columns_reg<(NRMAX >= 12 ? 12 : 8)>(Yb, m, j, j + 1, np, v, beta, norms);
        else if (NRMAX >= 16 && m - j <= 1024)
            reflect_columns_reg<(NRMAX >= 16 ? 16 : 8)>(Yb, m, j, j + 1, np, v, beta, norms);
        else
            reflect_columns(Yb, m, j, j + 1, np, v, beta, norms);
        if (tid == 0) {
            Yb[j + (long)j * m] = alpha;
            s_k = j + 1;
        }
        __syncthreads();
    }
    __syncthreads();
    const int k = s_k;
    if (tid == 0) kout[blockIdx.x] = k;
    for (int c = tid; c < np; c += kThreads) {
        perm[M.act + c] = pv[c];
        sr[M.act + c] = act[M.act + pv[c]];
    }
    id_coefficients(Yb, m, np, k, T64 + M.f, 0, np - k);
}

void launch_cpqr(int nbox, const BoxMeta* meta, double* Y, const int* act, int* sr, int* perm, int* k,
                 double* T64, double tol, double tie, int m_max, int np_max, hipStream_t s) {
    if (nbox == 0) return;
    size_t shm = (size_t)(np_max + m_max) * sizeof(double) + (size_t)np_max * sizeof(int);
    if (m_max <= 512)
        CBD_LAUNCH(k_cpqr<8>, dim3(nbox), dim3(kThreads), shm, s, meta, Y, act, sr, perm, k, T64, tol,
                           tie);
    else
        CBD_LAUNCH(k_cpqr<16>, dim3(nbox), dim3(kThreads), shm, s, meta, Y, act, sr, perm, k, T64, tol,
                           tie);
}

// Register-resident form for levels of many small boxes (at most 8 CPW columns and
// 64 NR rows): one 512-thread workgroup per box holds the whole matrix in registers
// (column q in wave q % 8, slot q / 8; lane l holds rows l + 64 t), so a pivot step
// moves no matrix data through memory.  Columns are never moved: their current
// positions are kept in LDS (pos, and inv for position -> column), which is all the
// tie rule needs.  Per step: the largest remaining norm and the lowest position
// within the tie window (two workgroup reductions); the pivot column's owner builds
// the reflector in LDS; every wave reflects its columns and recomputes their norms
// over the rows below the step.  The same arithmetic as k_cpqr per column (dot
// product, update, norm), with sums in a different order.  At the end the R rows
// 0 .. k-1 are written to Y in position order, and k, perm and sr as k_cpqr does;
// T comes from k_qr_coeff.
constexpr int kRegThreads = 512, kRegWaves = kRegThreads / 64;

template <int CPW, int NR>
__global__ __launch_bounds__(kRegThreads) void k_cpqr_reg(const BoxMeta* __restrict__ meta,
                                                          double* __restrict__ Y, const int* __restrict__ act,
                                                          int* __restrict__ sr, int* __restrict__ perm,
                                                          int* __restrict__ kout, double tol, double tie) {
    constexpr int kCols = kRegWaves * CPW, kRows = 64 * NR;
    __shared__ double nrm[kCols];
    __shared__ int pos[kCols], inv[kCols];
    __shared__ double vbuf[kRows];
    __shared__ double red[kRegWaves];
    __shared__ int redi[kRegWaves];
    __shared__ double s_beta;
    const BoxMeta M = meta[blockIdx.x];
    const int m = M.m, np = M.np;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double* Yb = Y + M.y;
    double col[CPW][NR];
    // load; norms of the full columns
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl) {
        const int q = sl * kRegWaves + w;
        double ss = 0.0;
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            const int r = lane + 64 * t;
            col[sl][t] = (q < np && r < m) ? Yb[r + (long)q * m] : 0.0;
            ss += col[sl][t] * col[sl][t];
        }
        ss = wave_sum(ss);
        if (lane == 0 && q < np) nrm[q] = sqrt(ss);
    }
    for (int q = tid; q < np; q += kRegThreads) {
        pos[q] = q;
        inv[q] = q;
    }
    for (int r = tid; r < kRows; r += kRegThreads) vbuf[r] = 0.0;
    __syncthreads();
    const int kmax = m < np ? m : np;
    double nu0 = 0.0;
    int k = 0;
    for (int j = 0; j < kmax; ++j) {
        // largest remaining norm (columns at positions >= j)
        double lm = 0.0;
        if (lane < CPW) {
            const int q = lane * kRegWaves + w;
            if (q < np && pos[q] >= j) lm = nrm[q];
        }
        lm = wave_max(lm);
        if (lane == 0) red[w] = lm;
        __syncthreads();
        double mx = red[0];
#pragma unroll
        for (int u = 1; u < kRegWaves; ++u) mx = red[u] > mx ? red[u] : mx;
        if (j == 0) nu0 = mx;
        if (nu0 == 0.0 || mx <= tol * nu0) break;     // uniform over the workgroup
        const double thr = mx - tie * nu0;
        int lp = INT_MAX;
        if (lane < CPW) {
            const int q = lane * kRegWaves + w;
            if (q < np && pos[q] >= j && nrm[q] >= thr) lp = pos[q];
        }
        lp = wave_min_int(lp);
        if (lane == 0) redi[w] = lp;
        __syncthreads();
        int pp = redi[0];
#pragma unroll
        for (int u = 1; u < kRegWaves; ++u) pp = redi[u] < pp ? redi[u] : pp;
        const int qp = inv[pp];                        // pivot column
        const int qj = inv[j];                         // column at position j
        const double xn = nrm[qp];
        // reflector of the pivot column, built by its owner wave into vbuf
        if (w == qp % kRegWaves) {
            const int sl = qp / kRegWaves;
            double x0 = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < CPW; ++s2)
                if (s2 == sl)
#pragma unroll
                    for (int t = 0; t < NR; ++t)
                        if (lane + 64 * t == j) x0 = col[s2][t];
            x0 = __shfl(x0, j & 63);
            // (the lane holding row j broadcast it; every lane of the wave now has x0)
            const double alpha = x0 >= 0.0 ? -xn : xn;
            const double vn2 = 2.0 * xn * xn + 2.0 * fabs(x0) * xn;
#pragma unroll
            for (int s2 = 0; s2 < CPW; ++s2)
                if (s2 == sl)
#pragma unroll
                    for (int t = 0; t < NR; ++t) {
                        const int r = lane + 64 * t;
                        if (r < kRows) vbuf[r] = r < j ? 0.0 : (r == j ? x0 - alpha : col[s2][t]);
                        if (r == j) col[s2][t] = alpha;
                        else if (r > j) col[s2][t] = 0.0;
                    }
            if (lane == 0) s_beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        }
        if (tid == 0) {
            pos[qj] = pp;
            inv[pp] = qj;
            pos[qp] = j;
            inv[j] = qp;
        }
        __syncthreads();
        const double beta = s_beta;
        double vr[NR];
#pragma unroll
        for (int t = 0; t < NR; ++t) vr[t] = vbuf[lane + 64 * t];
        // reflect every remaining column of this wave; norms over the rows below j
#pragma unroll
        for (int sl = 0; sl < CPW; ++sl) {
            const int q = sl * kRegWaves + w;
            if (q >= np || pos[q] <= j) continue;      // (uniform over the wave)
            double dt = 0.0;
#pragma unroll
            for (int t = 0; t < NR; ++t) dt = fma(vr[t], col[sl][t], dt);
            dt = wave_sum(dt) * beta;
            double ss = 0.0;
#pragma unroll
            for (int t = 0; t < NR; ++t) {
                col[sl][t] = fma(-dt, vr[t], col[sl][t]);
                const double y = lane + 64 * t > j ? col[sl][t] : 0.0;
                ss = fma(y, y, ss);
            }
            ss = wave_sum(ss);
            if (lane == 0) nrm[q] = sqrt(ss);
        }
        k = j + 1;
        __syncthreads();
    }
    // R rows 0 .. k-1 (in position order) back to Y; rank, column order, skeleton lists
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl) {
        const int q = sl * kRegWaves + w;
        if (q >= np) continue;
        const int c = pos[q];
#pragma unroll
        for (int t = 0; t < NR; ++t) {
            const int r = lane + 64 * t;
            if (r < k) Yb[r + (long)c * m] = col[sl][t];
        }
    }
    if (tid == 0) kout[blockIdx.x] = k;
    for (int c = tid; c < np; c += kRegThreads) {
        const int q = inv[c];
        perm[M.act + c] = q;
        sr[M.act + c] = act[M.act + q];
    }
}

bool cpqr_reg_fits(int m_max, int np_max) { return m_max <= 64 * 4 && np_max <= kRegWaves * 13; }

// Stepped form for levels with few, large boxes: one launch pair per pivot step
// (pivot + reflector: one workgroup per box; update: kQrCols columns per
// workgroup), so that all CUs share the reflections of the few boxes.  The
// state between launches lives in per-box device arrays (QrState).
constexpr int kQrCols = 16;

__global__ __launch_bounds__(kThreads) void k_qr_init(const BoxMeta* __restrict__ meta,
                                                      const double* __restrict__ Y, QrState st) {
    const BoxMeta M = meta[blockIdx.x];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int c0 = blockIdx.y * kQrCols;
    const int c1 = min(M.np, c0 + kQrCols);
    for (int c = c0 + wid; c < c1; c += kWaves) {
        const double* col = Y + M.y + (long)c * M.m;
        double q = 0;
        for (int r = lane; r < M.m; r += 64) q += col[r] * col[r];
        q = wave_sum(q);
        if (lane == 0) {
            st.norms[M.act + c] = sqrt(q);
            st.pv[M.act + c] = c;
        }
    }
    if (blockIdx.y == 0 && threadIdx.x == 0) {
        const int kmax = min(M.m, M.np);
        st.done[blockIdx.x] = kmax == 0;
        st.k[blockIdx.x] = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_qr_pivot(const BoxMeta* __restrict__ meta,
                                                       double* __restrict__ Y, QrState st, int j,
                                                       double tol, double tie) {
    __shared__ double red[kWaves];
    __shared__ int redi[kWaves];
    __shared__ double s_thr;
    __shared__ int s_stop, s_piv;
    const int b = blockIdx.x;
    if (st.done[b]) return;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int kmax = min(m, np);
    if (j >= kmax) {
        if (tid == 0) {
            st.done[b] = 1;
            st.k[b] = kmax;
        }
        return;
    }
    double* Yb = Y + M.y;
    double* norms = st.norms + M.act;
    double lmax = 0;
    for (int c = j + tid; c < np; c += kThreads) lmax = norms[c] > lmax ? norms[c] : lmax;
    lmax = wave_max(lmax);
    if (lane == 0) red[wid] = lmax;
    __syncthreads();
    if (tid == 0) {
        double mx = red[0];
        for (int w = 1; w < kWaves; ++w) mx = red[w] > mx ? red[w] : mx;
        if (j == 0) st.nu0[b] = mx;
        const double nu0 = j == 0 ? mx : st.nu0[b];
        s_stop = (nu0 == 0.0) || (mx <= tol * nu0);
        s_thr = mx - tie * nu0;
        if (s_stop) {
            st.done[b] = 1;
            st.k[b] = j;
        }
    }
    __syncthreads();
    if (s_stop) return;
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
    const double xn = norms[piv];
    if (piv != j) {
        double* cj = Yb + (long)j * m;
        double* cp = Yb + (long)piv * m;
        for (int r = tid; r < m; r += kThreads) {
            const double t = cj[r];
            cj[r] = cp[r];
            cp[r] = t;
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (piv != j) {
            int* pv = st.pv + M.act;
            const int t = pv[j];
            pv[j] = pv[piv];
            pv[piv] = t;
            norms[piv] = norms[j];
        }
        const double x0 = Yb[j + (long)j * m];
        const double alpha = x0 >= 0.0 ? -xn : xn;
        const double vn2 = 2.0 * xn * xn + 2.0 * fabs(x0) * xn;
        Yb[j + (long)j * m] = x0 - alpha;            // the reflector occupies column j
        st.alpha[M.act + j] = alpha;
        st.beta[b] = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    }
}

template <int NR>
__global__ __launch_bounds__(kThreads) void k_qr_update(const BoxMeta* __restrict__ meta,
                                                        double* __restrict__ Y, QrState st, int j) {
    extern __shared__ char smem_raw[];
    const int b = blockIdx.x;
    if (st.done[b]) return;
    const BoxMeta M = meta[b];
    const int c0 = max(j + 1, (int)blockIdx.y * kQrCols);
    const int c1 = min(M.np, (int)(blockIdx.y + 1) * kQrCols);
    if (c0 >= c1) return;
    double* Yb = Y + M.y;
    double* v = reinterpret_cast<double*>(smem_raw);
    for (int r = j + threadIdx.x; r < M.m; r += kThreads) v[r - j] = Yb[r + (long)j * M.m];
    __syncthreads();
    if constexpr (NR == 0)
        reflect_columns(Yb, M.m, j, c0, c1, v, st.beta[b], st.norms + M.act);
    else
        reflect_columns_reg<NR>(Yb, M.m, j, c0, c1, v, st.beta[b], st.norms + M.act);
}

__global__ __launch_bounds__(kThreads) void k_qr_finish(const BoxMeta* __restrict__ meta,
                                                        double* __restrict__ Y, QrState st,
                                                        const int* __restrict__ act, int* __restrict__ sr,
                                                        int* __restrict__ perm, int* __restrict__ kout) {
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int kmax = min(M.m, M.np);
    const int k = st.done[b] ? st.k[b] : kmax;
    double* Yb = Y + M.y;
    for (int j = threadIdx.x; j < k; j += kThreads) Yb[j + (long)j * M.m] = st.alpha[M.act + j];
    if (threadIdx.x == 0) kout[b] = k;
    for (int c = threadIdx.x; c < M.np; c += kThreads) {
        const int p = st.pv[M.act + c];
        perm[M.act + c] = p;
        sr[M.act + c] = act[M.act + p];
    }
}

// T = R11^{-1} R12 of the stepped boxes, kCoeffCols columns of T per workgroup.
constexpr int kCoeffCols = 64;
__global__ __launch_bounds__(kThreads) void k_qr_coeff(const BoxMeta* __restrict__ meta,
                                                       const double* __restrict__ Y, const int* __restrict__ kin,
                                                       double* __restrict__ T64) {
    const BoxMeta M = meta[blockIdx.x];
    const int k = kin[blockIdx.x];
    const int c_lo = blockIdx.y * kCoeffCols, c_hi = min(M.np - k, c_lo + kCoeffCols);
    if (c_lo >= c_hi) return;
    id_coefficients(Y + M.y, M.m, M.np, k, T64 + M.f, c_lo, c_hi);
}

void launch_qr_init(int nbox, int np_max, const BoxMeta* meta, const double* Y, const QrState& st,
                    hipStream_t s) {
    if (nbox == 0) return;
    CBD_LAUNCH(k_qr_init, dim3(nbox, (np_max + kQrCols - 1) / kQrCols), dim3(kThreads), 0, s, meta,
                       Y, st);
}
void launch_qr_step(int nbox, int np_max, int m_max, const BoxMeta* meta, double* Y, const QrState& st,
                    int j, double tol, double tie, hipStream_t s) {
    if (nbox == 0) return;
    CBD_LAUNCH(k_qr_pivot, dim3(nbox), dim3(kThreads), 0, s, meta, Y, st, j, tol, tie);
    // rows of the update: at most m_max - j; the register form holds up to 64 NR of them
    // (3072 rows; within 256 registers per lane)
    const int cb = (m_max - j + 63) / 64;
    const dim3 grid(nbox, (np_max + kQrCols - 1) / kQrCols);
    const size_t shm = (size_t)m_max * sizeof(double);
    if (cb <= 2)
        CBD_LAUNCH(k_qr_update<2>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 4)
        CBD_LAUNCH(k_qr_update<4>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 8)
        CBD_LAUNCH(k_qr_update<8>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 12)
        CBD_LAUNCH(k_qr_update<12>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 16)
        CBD_LAUNCH(k_qr_update<16>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 24)
        CBD_LAUNCH(k_qr_update<24>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 32)
        CBD_LAUNCH(k_qr_update<32>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else if (cb <= 48)
        CBD_LAUNCH(k_qr_update<48>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
    else
        CBD_LAUNCH(k_qr_update<0>, grid, dim3(kThreads), shm, s, meta, Y, st, j);
}
void launch_qr_finish(int nbox, int np_max, const BoxMeta* meta, double* Y, const QrState& st, const int* act,
                      int* sr, int* perm, int* k, double* T64, hipStream_t s) {
    if (nbox == 0) return;
    CBD_LAUNCH(k_qr_finish, dim3(nbox), dim3(kThreads), 0, s, meta, Y, st, act, sr, perm, k);
    CBD_LAUNCH(k_qr_coeff, dim3(nbox, (np_max + kCoeffCols - 1) / kCoeffCols), dim3(kThreads), 0, s,
                       meta, Y, k, T64);
}

void launch_cpqr_reg(int nbox, int np_max, int m_max, const BoxMeta* meta, double* Y, const int* act, int* sr,
                     int* perm, int* k, double* T64, double tol, double tie, hipStream_t s) {
    if (nbox == 0) return;
    // (up to 13 columns of 4 x 64 rows per wave: 104 registers of matrix, no spills)
    if (np_max <= kRegWaves * 8)
        CBD_LAUNCH((k_cpqr_reg<8, 4>), dim3(nbox), dim3(kRegThreads), 0, s, meta, Y, act, sr, perm, k, tol,
                           tie);
    else
        CBD_LAUNCH((k_cpqr_reg<13, 4>), dim3(nbox), dim3(kRegThreads), 0, s, meta, Y, act, sr, perm, k,
                           tol, tie);
    CBD_LAUNCH(k_qr_coeff, dim3(nbox, (np_max + kCoeffCols - 1) / kCoeffCols), dim3(kThreads), 0, s, meta,
                       Y, k, T64);
}

// ---- row compression of tall proxy matrices ---------------------------------
// Householder QR without pivoting, Y = Q R, by panels of kHqrPanel columns in
// the compact WY form H_1 ... H_w = I - V T V^T (T upper triangular).  Column
// norms of every trailing block, and with them the pivots, the stopping step and
// R11, R12 of the truncated pivoted QR, are invariant under Q^T, so the pivoted
// QR can run on the min(m, np) x np factor R instead of the m x np matrix Y.
// Reflectors: v_c = Y[c:, c] - alpha_c e_1 kept in place of column c (rows >= c),
// beta_c = 2 / ||v_c||^2, alpha_c (the diagonal of R) in a side array.  Each
// panel's reflectors are also written, zero-padded, to a per-box buffer in two
// layouts (Vc: m x kHqrPanel column-major; Vt: kHqrPanel x m) for the MFMA
// operands of the trailing update.
constexpr int kHqrPanel = 32;
static_assert(kHqrPanel * kHqrPanel == kHqrTw, "T slot size");

constexpr int kHqrThreads = 512;   // panel workgroup: more rows in flight per step
constexpr int kHqrWaves = kHqrThreads / 64;

// One workgroup per box.  Step jj: one pass over the panel rows computes, for
// every other panel column q, v_jj . Y[:, j0+q] (q < jj: a column of the Gram
// matrix of the reflectors, for T; q > jj: the reflection coefficients); a
// second pass applies the reflection and accumulates the next column's norm.
__global__ __launch_bounds__(kHqrThreads) void k_hqr_panel(const BoxMeta* __restrict__ meta, double* __restrict__ Y,
                                                        int j0, double* __restrict__ Tw,
                                                        double* __restrict__ alpha, double* __restrict__ Vbuf,
                                                        long vstride) {
    __shared__ double red[kHqrPanel][kHqrWaves];
    __shared__ double s_sc[kHqrPanel];
    __shared__ double s_T[kHqrPanel * kHqrPanel];
    __shared__ double s_xn2;
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np, kmax = min(m, np);
    if (j0 >= kmax) return;
    const int w = min(kHqrPanel, kmax - j0);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double* Yb = Y + M.y;
    double* P = Yb + (long)j0 * m;          // panel column q at P + q * m
    for (int e = tid; e < kHqrPanel * kHqrPanel; e += kHqrThreads) s_T[e] = 0.0;
    // norm^2 of the first column over rows j0..
    {
        double q = 0.0;
        for (int r = j0 + tid; r < m; r += kHqrThreads) q += P[r] * P[r];
        q = wave_sum(q);
        if (lane == 0) red[0][wid] = q;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int v = 0; v < kHqrWaves; ++v) t += red[0][v];
            s_xn2 = t;
        }
        __syncthreads();
    }
    for (int jj = 0; jj < w; ++jj) {
        const int c = j0 + jj;
        double* vc = P + (long)jj * m;
        // reflector of column c
        if (tid == 0) {
            const double xn = sqrt(s_xn2);
            const double x0 = vc[c];
            const double al = x0 >= 0.0 ? -xn : xn;
            const double vn2 = 2.0 * xn * xn + 2.0 * fabs(x0) * xn;
            const double beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
            vc[c] = x0 - al;
            alpha[M.act + c] = al;
            s_T[jj + jj * kHqrPanel] = beta;
        }
        __syncthreads();
        // pass 1: v . Y[:, j0 + q] for every panel column q != jj (rows c..).  All
        // loads are unconditional (column index clamped into the panel) so that they
        // are in flight together; the unused products are masked.
        double part[kHqrPanel];
#pragma unroll
        for (int q = 0; q < kHqrPanel; ++q) part[q] = 0.0;
        for (int r = c + tid; r < m; r += kHqrThreads) {
            const double v = vc[r];
            double y[kHqrPanel];
#pragma unroll
            for (int q = 0; q < kHqrPanel; ++q) y[q] = P[r + (long)min(q, w - 1) * m];
#pragma unroll
            for (int q = 0; q < kHqrPanel; ++q) part[q] += (q != jj && q < w) ? v * y[q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kHqrPanel; ++q) {
            if (q == jj || q >= w) continue;
            const double t = wave_sum(part[q]);
            if (lane == 0) red[q][wid] = t;
        }
        __syncthreads();
        const double beta = s_T[jj + jj * kHqrPanel];
        if (tid < w && tid != jj) {
            double t = 0.0;
            for (int v = 0; v < kHqrWaves; ++v) t += red[tid][v];
            s_sc[tid] = tid > jj ? beta * t : t;     // reflection coefficient, or Gram entry G[tid][jj]
        }
        __syncthreads();
        // T[0:jj, jj] = -beta T[0:jj, 0:jj] G[0:jj, jj]
        if (tid < jj) {
            double t = 0.0;
            for (int a2 = tid; a2 < jj; ++a2) t += s_T[tid + a2 * kHqrPanel] * s_sc[a2];
            s_T[tid + jj * kHqrPanel] = -beta * t;
        }
        // pass 2: Y[:, j0 + q] -= s_q v for q > jj (rows c..), and the next column's
        // norm; loads clamped to the columns jj+1..w-1 as in pass 1
        double nx = 0.0;
        if (jj + 1 < w) {
            for (int r = c + tid; r < m; r += kHqrThreads) {
                const double v = vc[r];
                double y[kHqrPanel];
#pragma unroll
                for (int q = 0; q < kHqrPanel; ++q) y[q] = P[r + (long)min(max(q, jj + 1), w - 1) * m];
#pragma unroll
                for (int q = 0; q < kHqrPanel; ++q) {
                    if (q <= jj || q >= w) continue;
                    const double yn = y[q] - s_sc[q] * v;
                    P[r + (long)q * m] = yn;
                    if (q == jj + 1 && r > c) nx += yn * yn;
                }
            }
        }
        nx = wave_sum(nx);
        if (lane == 0) red[0][wid] = nx;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int v = 0; v < kHqrWaves; ++v) t += red[0][v];
            s_xn2 = t;
        }
        __syncthreads();
    }
    double* Tb = Tw + (long)b * kHqrTw;
    for (int e = tid; e < kHqrPanel * kHqrPanel; e += kHqrThreads) Tb[e] = s_T[e];
    // zero-padded reflectors in both layouts (rows j0..m-1)
    double* Vc = Vbuf + (long)b * vstride;
    double* Vt = Vc + (long)m * kHqrPanel;
    for (long e = tid; e < (long)(m - j0) * kHqrPanel; e += kHqrThreads) {
        const int r = j0 + (int)(e % (m - j0)), a = (int)(e / (m - j0));
        const double v = (a < w && r >= j0 + a) ? P[r + (long)a * m] : 0.0;
        Vc[r + (long)a * m] = v;
    }
    for (long e = tid; e < (long)(m - j0) * kHqrPanel; e += kHqrThreads) {
        const int a = (int)(e % kHqrPanel), r = j0 + (int)(e / kHqrPanel);
        const double v = (a < w && r >= j0 + a) ? P[r + (long)a * m] : 0.0;
        Vt[a + (long)r * kHqrPanel] = v;
    }
}

// Register-resident panel for matrices of at most 512 * RR rows below j0: every
// thread keeps rows j0 + tid + 512 i (i < RR) of the kHqrRegW panel columns in
// registers, so that a step costs two workgroup reductions and no memory pass.
// Same reflectors, T and outputs as k_hqr_panel (panel width kHqrRegW).
constexpr int kHqrRegW = 16;
constexpr int kHqrRegThreads = 512;

template <int RR>
__global__ __launch_bounds__(kHqrRegThreads) void k_hqr_panel_reg(const BoxMeta* __restrict__ meta,
                                                                  double* __restrict__ Y, int j0,
                                                                  double* __restrict__ Tw,
                                                                  double* __restrict__ alpha,
                                                                  double* __restrict__ Vbuf, long vstride) {
    constexpr int W = kHqrRegW, NW = kHqrRegThreads / 64;
    __shared__ double red[W][NW];
    __shared__ double s_sc[W];
    __shared__ double s_T[kHqrPanel * kHqrPanel];
    __shared__ double s_xn2;
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np, kmax = min(m, np);
    if (j0 >= kmax) return;
    const int w = min(W, kmax - j0);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double* P = Y + M.y + (long)j0 * m;      // panel column q at P + q * m
    for (int e = tid; e < kHqrPanel * kHqrPanel; e += kHqrRegThreads) s_T[e] = 0.0;
    double y[RR][W];
#pragma unroll
    for (int i = 0; i < RR; ++i) {
        const int r = j0 + tid + kHqrRegThreads * i;
        const int rc = min(r, m - 1);
#pragma unroll
        for (int q = 0; q < W; ++q) y[i][q] = P[rc + (long)min(q, w - 1) * m];
#pragma unroll
        for (int q = 0; q < W; ++q) y[i][q] = (r < m && q < w) ? y[i][q] : 0.0;
    }
    auto block_sum = [&](double v, int slot) {
        v = wave_sum(v);
        if (lane == 0) red[slot][wid] = v;
    };
    {
        double q0 = 0.0;
#pragma unroll
        for (int i = 0; i < RR; ++i) q0 += y[i][0] * y[i][0];
        block_sum(q0, 0);
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int v = 0; v < NW; ++v) t += red[0][v];
            s_xn2 = t;
        }
        __syncthreads();
    }
    for (int jj = 0; jj < w; ++jj) {
        const int c = j0 + jj;
        // row c is row slot 0 of thread jj
        if (tid == jj) {
            double x0 = 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q) x0 = q == jj ? y[0][q] : x0;
            const double xn = sqrt(s_xn2);
            const double al = x0 >= 0.0 ? -xn : xn;
            const double vn2 = 2.0 * xn * xn + 2.0 * fabs(x0) * xn;
            const double beta = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q)
                if (q == jj) y[0][q] = x0 - al;
            alpha[M.act + c] = al;
            s_T[jj + jj * kHqrPanel] = beta;
        }
        __syncthreads();
        double v[RR];
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            const int r = j0 + tid + kHqrRegThreads * i;
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < W; ++q) t = q == jj ? y[i][q] : t;
            v[i] = r >= c ? t : 0.0;
        }
        // v . column q for every q != jj: Gram column (q < jj) or reflection coefficient (q > jj)
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q == jj || q >= w) continue;
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < RR; ++i) t += v[i] * y[i][q];
            block_sum(t, q);
        }
        __syncthreads();
        const double beta = s_T[jj + jj * kHqrPanel];
        if (tid < w && tid != jj) {
            double t = 0.0;
            for (int u = 0; u < NW; ++u) t += red[tid][u];
            s_sc[tid] = tid > jj ? beta * t : t;
        }
        __syncthreads();
        if (tid < jj) {
            double t = 0.0;
            for (int a2 = tid; a2 < jj; ++a2) t += s_T[tid + a2 * kHqrPanel] * s_sc[a2];
            s_T[tid + jj * kHqrPanel] = -beta * t;
        }
        // reflection of the columns q > jj, and the next column's norm (rows > c)
        double nx = 0.0;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q <= jj || q >= w) continue;
            const double sq = s_sc[q];
#pragma unroll
            for (int i = 0; i < RR; ++i) y[i][q] -= sq * v[i];
            if (q == jj + 1) {
#pragma unroll
                for (int i = 0; i < RR; ++i) {
                    const int r = j0 + tid + kHqrRegThreads * i;
                    if (r > c) nx += y[i][q] * y[i][q];
                }
            }
        }
        block_sum(nx, 0);
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int u = 0; u < NW; ++u) t += red[0][u];
            s_xn2 = t;
        }
        __syncthreads();
    }
    // panel back to Y, reflectors (zero-padded to kHqrPanel columns) to the staging buffer
    double* Vc = Vbuf + (long)b * vstride;
    double* Vt = Vc + (long)m * kHqrPanel;
#pragma unroll
    for (int i = 0; i < RR; ++i) {
        const int r = j0 + tid + kHqrRegThreads * i;
        if (r >= m) continue;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            if (q >= w) continue;
            P[r + (long)q * m] = y[i][q];
        }
#pragma unroll
        for (int a = 0; a < kHqrPanel; ++a) {
            double vv = 0.0;
            if (a < W) vv = (a < w && r >= j0 + a) ? y[i][a < W ? a : 0] : 0.0;
            Vc[r + (long)a * m] = vv;
            Vt[a + (long)r * kHqrPanel] = vv;
        }
    }
    double* Tb = Tw + (long)b * kHqrTw;
    for (int e = tid; e < kHqrPanel * kHqrPanel; e += kHqrRegThreads) Tb[e] = s_T[e];
}

// Trailing columns c >= j0 + w, 16 per workgroup: A <- A - V (T^T (V^T A)), both
// products on FP64 MFMA (v_mfma_f64_16x16x4f64).  W = V^T A splits its rows over
// the waves; A - V W' takes 16-row tiles per wave.
__global__ __launch_bounds__(kThreads) void k_hqr_update(const BoxMeta* __restrict__ meta, double* __restrict__ Y,
                                                         int j0, int pw, const double* __restrict__ Tw,
                                                         const double* __restrict__ Vbuf, long vstride) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ double s_T[kHqrPanel * kHqrPanel];
    __shared__ double s_P[kWaves][kHqrPanel * 16];
    __shared__ double s_W[kHqrPanel * 16];
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np, kmax = min(m, np);
    if (j0 >= kmax) return;
    const int w = min(pw, kmax - j0);
    const int c0 = (int)blockIdx.y * 16;
    const int lo = max(j0 + w, c0), hi = min(np, c0 + 16);
    if (lo >= hi) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    double* Yb = Y + M.y;
    const double* Vc = Vbuf + (long)b * vstride;
    const double* Vt = Vc + (long)m * kHqrPanel;
    const double* Tb = Tw + (long)b * kHqrTw;
    for (int e = tid; e < kHqrPanel * kHqrPanel; e += kThreads) s_T[e] = Tb[e];
    const int col = c0 + li;
    const bool cin = col >= lo && col < hi;
    const double* ycol = Yb + (long)(cin ? col : lo) * m;
    // W = V^T A: rows j0.. in 4-row steps, step s on wave s % kWaves
    // (reflectors w..31 are zero: a panel of at most 16 skips the second half)
    const bool two = w > 16;
    v4 w0 = {0, 0, 0, 0}, w1 = {0, 0, 0, 0};
    for (int r0 = j0 + 4 * wid; r0 < m; r0 += 4 * kWaves) {
        const int r = r0 + lk;
        const bool rin = r < m;
        const double a0 = rin ? Vt[li + (long)r * kHqrPanel] : 0.0;
        const double bb = (rin && cin) ? ycol[r] : 0.0;
        w0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb, w0, 0, 0, 0);
        if (two) {
            const double a1 = rin ? Vt[16 + li + (long)r * kHqrPanel] : 0.0;
            w1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb, w1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int a = 4 * v + lk;            // accumulator row
        s_P[wid][a + li * kHqrPanel] = w0[v];
        s_P[wid][16 + a + li * kHqrPanel] = w1[v];
    }
    __syncthreads();
    for (int e = tid; e < kHqrPanel * 16; e += kThreads) {
        double t = 0.0;
        for (int v = 0; v < kWaves; ++v) t += s_P[v][e];
        s_W[e] = t;
    }
    __syncthreads();
    // W' = -T^T W (T upper triangular: row a of T^T has entries a2 <= a), into s_P[0]
    for (int e = tid; e < kHqrPanel * 16; e += kThreads) {
        const int a = e % kHqrPanel, cc = e / kHqrPanel;
        double t = 0.0;
        for (int a2 = 0; a2 <= a; ++a2) t += s_T[a2 + a * kHqrPanel] * s_W[a2 + cc * kHqrPanel];
        s_P[0][e] = -t;
    }
    __syncthreads();
    // A += V W' over 16-row tiles (rows j0..m-1)
    const double* Wn = s_P[0];
    for (int t0 = j0 + 16 * wid; t0 < m; t0 += 16 * kWaves) {
        v4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = t0 + 4 * v + lk;
            acc[v] = (r < m && cin) ? ycol[r] : 0.0;
        }
        const int ra = t0 + li;
#pragma unroll
        for (int ks = 0; ks < kHqrPanel / 8; ++ks) {
            const int a = 4 * ks + lk;
            const double av = ra < m ? Vc[ra + (long)a * m] : 0.0;
            const double bv = Wn[a + li * kHqrPanel];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        if (two) {
#pragma unroll
            for (int ks = kHqrPanel / 8; ks < kHqrPanel / 4; ++ks) {
                const int a = 4 * ks + lk;
                const double av = ra < m ? Vc[ra + (long)a * m] : 0.0;
                const double bv = Wn[a + li * kHqrPanel];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
        }
        if (cin) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = t0 + 4 * v + lk;
                if (r < m) Yb[r + (long)col * m] = acc[v];
            }
        }
    }
}

// R (min(m, np) x np, zero below the diagonal) of every box into the compact
// layout of cmeta (cmeta[b].y; cmeta[b].m = min(m, np)).
__global__ __launch_bounds__(kThreads) void k_hqr_compact(const BoxMeta* __restrict__ meta,
                                                          const double* __restrict__ Y,
                                                          const double* __restrict__ alpha,
                                                          const BoxMeta* __restrict__ cmeta,
                                                          double* __restrict__ Rc) {
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int mr = cmeta[b].m;
    const double* Yb = Y + M.y;
    double* Rb = Rc + cmeta[b].y;
    for (long e = (long)blockIdx.y * kThreads + threadIdx.x; e < (long)mr * M.np; e += (long)gridDim.y * kThreads) {
        const int r = (int)(e % mr), c = (int)(e / mr);
        Rb[e] = r < c ? Yb[r + (long)c * M.m] : (r == c ? alpha[M.act + c] : 0.0);
    }
}

void launch_hqr(int nbox, int np_max, int m_max, int k_max, const BoxMeta* meta, double* Y, double* Tw,
                double* alpha, double* Vbuf, const BoxMeta* cmeta, double* Rc, hipStream_t s) {
    if (nbox == 0) return;
    const long vstride = 2L * m_max * kHqrPanel;
    const int ct = (np_max + 15) / 16;
    // panels held in registers when every matrix has at most 2560 rows
    const int rr = (m_max + kHqrRegThreads - 1) / kHqrRegThreads;
    const int pw = rr <= 5 ? kHqrRegW : kHqrPanel;
    for (int j0 = 0; j0 < k_max; j0 += pw) {
        if (rr <= 2)
            CBD_LAUNCH(k_hqr_panel_reg<2>, dim3(nbox), dim3(kHqrRegThreads), 0, s, meta, Y, j0, Tw, alpha,
                               Vbuf, vstride);
        else if (rr == 3)
            CBD_LAUNCH(k_hqr_panel_reg<3>, dim3(nbox), dim3(kHqrRegThreads), 0, s, meta, Y, j0, Tw, alpha,
                               Vbuf, vstride);
        else if (rr <= 5)
            CBD_LAUNCH(k_hqr_panel_reg<5>, dim3(nbox), dim3(kHqrRegThreads), 0, s, meta, Y, j0, Tw, alpha,
                               Vbuf, vstride);
        else
            CBD_LAUNCH(k_hqr_panel, dim3(nbox), dim3(kHqrThreads), 0, s, meta, Y, j0, Tw, alpha, Vbuf,
                               vstride);
        if (j0 + pw < np_max)
            CBD_LAUNCH(k_hqr_update, dim3(nbox, ct), dim3(kThreads), 0, s, meta, Y, j0, pw, Tw, Vbuf,
                               vstride);
    }
    CBD_LAUNCH(k_hqr_compact, dim3(nbox, 16), dim3(kThreads), 0, s, meta, Y, alpha, cmeta, Rc);
}

// ---- randomized ID: the sketch Z = Omega Y -----------------------------------
// Omega (ell x m per box) holds random signs from a counter-based hash: the
// splitmix64 output function of seed + key * G1 + i * G2 + rowkey * G3 (mod 2^64),
// top bit 0 -> +1, 1 -> -1; key = (subdomain << 40) | (level << 32) | box, rowkey =
// global index of a near-field row's point, N + q for proxy row q.  Z (ell x np,
// column-major) on FP64 MFMA: each wave one 16 x 16 tile of Z, the sign operand
// generated per lane, Y read as the B operand.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The signs of Omega, one bit each: word w of row `row` of box b holds the signs of
// sketch rows 32 w .. 32 w + 31 for that row of Y (bit u: 1 for -1), at
// bits + boff[b] + row * nw + w, nw = ceil(ell / 32).  One thread per word.
__global__ __launch_bounds__(kThreads) void k_sketch_signs(const BoxMeta* __restrict__ meta,
                                                           const BoxMeta* __restrict__ zmeta,
                                                           const int* __restrict__ nearl,
                                                           const int* __restrict__ cidx, long N,
                                                           unsigned long long seed,
                                                           const unsigned long long* __restrict__ keys,
                                                           const long* __restrict__ boff,
                                                           unsigned* __restrict__ bits) {
    const int b = blockIdx.x;
    const int ell = zmeta[b].m;
    if (ell == 0) return;
    const BoxMeta M = meta[b];
    const int nw = (ell + 31) >> 5;
    const long e = (long)blockIdx.y * kThreads + threadIdx.x;
    if (e >= (long)M.m * nw) return;
    const int row = (int)(e / nw), wd = (int)(e % nw);
    const unsigned long long rk =
        row < M.nnear ? (unsigned long long)cidx[nearl[M.near + row]] : (unsigned long long)(N + (row - M.nnear));
    const unsigned long long base = seed + keys[b] * 0x9E3779B97F4A7C15ull + rk * 0x8CB92BA72F3D8DD7ull;
    unsigned hw = 0;
    for (int u = 0; u < 32; ++u) {
        const int i = wd * 32 + u;
        if (i < ell) {
            const unsigned long long h = mix64(base + (unsigned long long)i * 0xD1B54A32D192ED03ull);
            hw |= (unsigned)(h >> 63) << u;
        }
    }
    bits[boff[b] + e] = hw;
}

// Z = Omega Y on FP64 MFMA.  A workgroup computes a tile of Z of kWaves * 16 * RBW
// sketch rows and C columns (wave w: RBW row blocks of 16 of it, C / 16
// accumulators each); a taller tile reads Y fewer times (Y is read once per tile
// row).  Rows of Y stream through LDS in chunks of kSkK (coalesced column segments)
// with the tile's sign words for them; each lane expands its A operand from a bit.
// The next chunk's loads are issued before the current chunk is multiplied.  Every
// entry of Z sums over the rows in steps of four in ascending order; rows of Z past
// ell are computed and dropped.
constexpr int kSkK = 32;
template <int RBW, int C>
__global__ __launch_bounds__(kThreads) void k_sketch(const BoxMeta* __restrict__ meta,
                                                     const BoxMeta* __restrict__ zmeta,
                                                     const double* __restrict__ Y,
                                                     const long* __restrict__ boff,
                                                     const unsigned* __restrict__ bits,
                                                     double* __restrict__ Z, int ti) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    constexpr int I = kWaves * 16 * RBW;   // sketch rows per workgroup
    constexpr int NW = I / 32;             // sign words per Y row of the tile
    constexpr int LdB = C + 1;
    constexpr int QY = C / 8;              // Y values staged per thread
    __shared__ double sB[kSkK * LdB];
    __shared__ unsigned sW[kSkK * NW];
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int ell = zmeta[b].m, np = M.np, m = M.m;
    const int i0 = (int)(blockIdx.y % ti) * I, c0 = (int)(blockIdx.y / ti) * C;
    if (ell == 0 || i0 >= ell || c0 >= np) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    v4 acc[RBW][C / 16];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int t = 0; t < C / 16; ++t) acc[rb][t] = v4{0, 0, 0, 0};
    // staging roles: chunk row sr of Y columns w C/4 + (lane >> 5) + 2 q; sign word u of
    // chunk row kw (threads below kSkK * NW)
    const int sr = lane & 31, sc0 = w * (C / 4) + (lane >> 5);
    const double* Ybox = Y + M.y;
    const int nw = (ell + 31) >> 5;
    const int kw = tid / NW, u = tid % NW;
    const bool wrole = tid < kSkK * NW && (i0 >> 5) + u < nw;
    const unsigned* wsrc = bits + boff[b] + (i0 >> 5) + u;
    double yv[QY];
    unsigned sw = 0;
    auto fetch = [&](int k) {
#pragma unroll
        for (int q = 0; q < QY; ++q)
            yv[q] = Ybox[(long)min(c0 + sc0 + 2 * q, np - 1) * m + min(k + sr, m - 1)];
        if (wrole) sw = wsrc[(long)min(k + kw, m - 1) * nw];
    };
    fetch(0);
    for (int k0 = 0; k0 < m; k0 += kSkK) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QY; ++q) {
            const int cc = sc0 + 2 * q;
            sB[sr * LdB + cc] = (c0 + cc < np && k0 + sr < m) ? yv[q] : 0.0;
        }
        if (tid < kSkK * NW) sW[tid] = wrole ? sw : 0u;
        __syncthreads();
        if (k0 + kSkK < m) fetch(k0 + kSkK);
#pragma unroll 2
        for (int ks = 0; ks < kSkK / 4; ++ks) {
            const int kk = ks * 4 + lk;
            double a[RBW];
#pragma unroll
            for (int rb = 0; rb < RBW; ++rb) {
                const int r = w * 16 * RBW + rb * 16 + li;   // sketch row within the tile
                a[rb] = ((sW[kk * NW + (r >> 5)] >> (r & 31)) & 1u) ? -1.0 : 1.0;
            }
#pragma unroll
            for (int t = 0; t < C / 16; ++t) {
                const double bv = sB[kk * LdB + t * 16 + li];
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb)
                    acc[rb][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], bv, acc[rb][t], 0, 0, 0);
            }
        }
    }
    double* Zb = Z + zmeta[b].y;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int t = 0; t < C / 16; ++t) {
            const int c = c0 + t * 16 + li;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = i0 + w * 16 * RBW + rb * 16 + 4 * v + lk;
                if (ii < ell && c < np) Zb[ii + (long)c * ell] = acc[rb][t][v];
            }
        }
}

void launch_sketch(int nbox, int np_max, long mw_max, const BoxMeta* meta, const BoxMeta* zmeta, const double* Y,
                   const int* nearl, const int* cidx, long N, unsigned long long seed,
                   const unsigned long long* keys, const long* boff, unsigned* bits, double* Z, hipStream_t s) {
    if (nbox == 0) return;
    CBD_LAUNCH(k_sketch_signs, dim3(nbox, (unsigned)((mw_max + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       s, meta, zmeta, nearl, cidx, N, seed, keys, boff, bits);
    // ell < np for every sketched box, so np_max bounds both dimensions of Z
    constexpr int RBW = 2, C = 128, I = kWaves * 16 * RBW;
    const int ti = (np_max + I - 1) / I, tc = (np_max + C - 1) / C;
    CBD_LAUNCH((k_sketch<RBW, C>), dim3(nbox, ti * tc), dim3(kThreads), 0, s, meta, zmeta, Y, boff, bits, Z,
                       ti);
}

// ---- box matrix A_pp --------------------------------------------------------
// Boxes made of grid points take kernel entries; a parent box takes its
// children's B_ss on the diagonal blocks and kernel entries between children.
// Workgroup (box, y) fills columns [c_lo, c_hi) of its box.  Columns and rows are
// staged in LDS in chunks of kBm (grid index, coordinates, column weight or row scale,
// child reference); then every thread takes entries of the chunk pair, rows fastest,
// so the writes run down the column-major A and no thread waits on a global load.
template <int D, typename R>
__global__ __launch_bounds__(kThreads) void k_box_matrix(ProblemView P,
                                                         const BoxMeta* __restrict__ meta,
                                                         const int* __restrict__ act,
                                                         const int* __restrict__ cidx,
                                                         const ChildRef<R>* __restrict__ ch,
                                                         R* __restrict__ App) {
    constexpr int kBm = 256;
    __shared__ double rx[D][kBm], rsc[kBm], cx[D][kBm], cw[kBm];
    __shared__ long rgi[kBm], cgi[kBm];
    __shared__ ChildRef<R> rref[kBm], cref[kBm];
    const BoxMeta M = meta[blockIdx.x];
    const int np = M.np;
    const int per = (np + gridDim.y - 1) / gridDim.y;
    const int c_lo = blockIdx.y * per, c_hi = min(np, c_lo + per);
    if (c_lo >= c_hi) return;
    const int tid = threadIdx.x;
    const bool parent = M.ch >= 0;
    R* A = App + M.app;
    for (int cb = c_lo; cb < c_hi; cb += kBm) {
        const int ncol = min(kBm, c_hi - cb);
        __syncthreads();
        for (int i = tid; i < ncol; i += kThreads) {
            const long gj = cidx[act[M.act + cb + i]];
#pragma unroll
            for (int t = 0; t < D; ++t) cx[t][i] = P.pts[t * P.N + gj];
            cw[i] = P.w[gj];
            cgi[i] = gj;
            if (parent) cref[i] = ch[M.ch + cb + i];
        }
        for (int r0 = 0; r0 < np; r0 += kBm) {
            const int nrow = min(kBm, np - r0);
            if (r0 > 0) __syncthreads();
            for (int i = tid; i < nrow; i += kThreads) {
                const long gi = cidx[act[M.act + r0 + i]];
#pragma unroll
                for (int t = 0; t < D; ++t) rx[t][i] = P.pts[t * P.N + gi];
                rsc[i] = P.rs[gi];
                rgi[i] = gi;
                if (parent) rref[i] = ch[M.ch + r0 + i];
            }
            __syncthreads();
            for (int e = tid; e < nrow * ncol; e += kThreads) {
                const int rr = e % nrow, cc = e / nrow;
                R val;
                if (parent && rref[rr].bss == cref[cc].bss) {
                    val = rref[rr].bss[rref[rr].pos + (long)cref[cc].pos * rref[rr].ldk];
                } else if (rgi[rr] == cgi[cc]) {
                    val = (R)P.diag[cgi[cc]];
                } else {
                    double r2 = 0.0;
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const double dx = rx[t][rr] - cx[t][cc];
                        r2 += dx * dx;
                    }
                    val = (R)(rsc[rr] * laplace_from_r2<D>(r2) * cw[cc]);
                }
                A[(long)(cb + cc) * np + r0 + rr] = val;
            }
        }
    }
}

template <typename R>
void launch_box_matrix(const ProblemView& P, int nbox, int np_max, const BoxMeta* meta, const int* act,
                       const int* cidx, const ChildRef<R>* ch, R* App, hipStream_t s) {
    if (nbox == 0) return;
    // workgroups per box: about 4096 entries each, at most 16, or more when the level has
    // few boxes (up to about 1024 workgroups in all)
    const int cap = std::min(256, std::max(16, 1024 / nbox));
    dim3 grid(nbox, std::max(1, std::min(cap, (int)(((long)np_max * np_max + 4095) / 4096))));
    if (P.d == 2)
        CBD_LAUNCH((k_box_matrix<2, R>), grid, dim3(kThreads), 0, s, P, meta, act, cidx, ch,
                           App);
    else
        CBD_LAUNCH((k_box_matrix<3, R>), grid, dim3(kThreads), 0, s, P, meta, act, cidx, ch,
                           App);
}

// ---- workgroup-level MFMA GEMM ----------------------------------------------
// Matrix-core instruction per precision: v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32
// (A: lane l holds row l%16, k l/16; B: column l%16, k l/16).  The accumulator
// layouts differ (checked with an in-bounds probe): register v of lane l holds
// row 4v + l/16 (f64) or 4(l/16) + v (f32) of column l%16.
template <typename R>
struct Mma;
template <>
struct Mma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int v, int lane) { return 4 * v + (lane >> 4); }
};
template <>
struct Mma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int v, int lane) { return 4 * (lane >> 4) + v; }
};

// One 64 x 64 tile (rows i0.., columns j0..) of C = beta C_in + alpha op(A) op(B),
// computed by the whole workgroup: k runs in chunks of kBgK through LDS (op(A) and
// op(B) stored k-major, each loaded along its contiguous direction), wave w takes
// the 32 x 32 quadrant (w & 1, w >> 1) as 2 x 2 MFMA tiles.  Every entry sums over
// k in steps of four in ascending order, as tile_gemm does.  With upper set, the
// 16 x 16 tiles entirely below the diagonal are not written.  Ends with a barrier.
constexpr int kBgK = 32;
template <typename R>
struct BgShared {
    R a[kBgK][64 + 16];   // row stride 80: the operand reads of a wave fall in distinct banks
    R b[kBgK][64 + 16];
};

template <typename R, bool ta, bool tb>
__device__ void block_gemm64(BgShared<R>& sh, int i0, int j0, int M, int N, int K, R alpha, const R* A, int lda,
                             const R* B, int ldb, R beta, const R* Cin, R* C, int ldc, bool upper) {
    typedef typename Mma<R>::v4 v4;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
    v4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = v4{0, 0, 0, 0};
    // staging: along the contiguous direction of each operand
    //   rows-contiguous (A untransposed, B transposed): index x = tid % 64, k = tid / 64 + 4 q
    //   k-contiguous (A transposed, B untransposed):   k = tid % 32, index x = tid / 32 + 8 q
    for (int k0 = 0; k0 < K; k0 += kBgK) {
        R ra[8], rb[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int x, kk;
            if (!ta) { x = tid & 63; kk = (tid >> 6) + 4 * q; } else { kk = tid & 31; x = (tid >> 5) + 8 * q; }
            const int gi = min(i0 + x, M - 1), gk = min(k0 + kk, K - 1);
            ra[q] = ta ? A[gk + (long)gi * lda] : A[gi + (long)gk * lda];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int x, kk;
            if (tb) { x = tid & 63; kk = (tid >> 6) + 4 * q; } else { kk = tid & 31; x = (tid >> 5) + 8 * q; }
            const int gj = min(j0 + x, N - 1), gk = min(k0 + kk, K - 1);
            rb[q] = tb ? B[gj + (long)gk * ldb] : B[gk + (long)gj * ldb];
        }
        __syncthreads();   // the previous chunk's operands are no longer read
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int x, kk;
            if (!ta) { x = tid & 63; kk = (tid >> 6) + 4 * q; } else { kk = tid & 31; x = (tid >> 5) + 8 * q; }
            sh.a[kk][x] = (i0 + x < M && k0 + kk < K) ? ra[q] : (R)0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int x, kk;
            if (tb) { x = tid & 63; kk = (tid >> 6) + 4 * q; } else { kk = tid & 31; x = (tid >> 5) + 8 * q; }
            sh.b[kk][x] = (j0 + x < N && k0 + kk < K) ? rb[q] : (R)0;
        }
        __syncthreads();
        const int ks_end = min(kBgK, K - k0);
        for (int ks = 0; ks < ks_end; ks += 4) {
            const int kk = ks + lk;
            const R a0 = sh.a[kk][wi + li], a1 = sh.a[kk][wi + 16 + li];
            const R b0 = sh.b[kk][wj + li], b1 = sh.b[kk][wj + 16 + li];
            acc[0][0] = Mma<R>::op(a0, b0, acc[0][0]);
            acc[0][1] = Mma<R>::op(a0, b1, acc[0][1]);
            acc[1][0] = Mma<R>::op(a1, b0, acc[1][0]);
            acc[1][1] = Mma<R>::op(a1, b1, acc[1][1]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int ti0 = i0 + wi + 16 * a, tj0 = j0 + wj + 16 * c;
            if (upper && ti0 > tj0 + 15) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = ti0 + Mma<R>::row(v, lane), jj = tj0 + li;
                if (ii < M && jj < N) {
                    const long o = ii + (long)jj * ldc;
                    C[o] = (beta == (R)0 ? (R)0 : beta * Cin[o]) + alpha * acc[a][c][v];
                }
            }
        }
    __syncthreads();
}

// One 16 x 16 tile (rows i0.., columns j0..) of C = beta C_in + alpha op(A) op(B),
// computed by one wave; C_in may be C itself.
template <typename R>
__device__ __forceinline__ void tile_gemm(int i0, int j0, int M, int N, int K, R alpha, const R* A, int lda,
                                          bool ta, const R* B, int ldb, bool tb, R beta, const R* Cin, R* C,
                                          int ldc) {
    typedef typename Mma<R>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    v4 acc = {0, 0, 0, 0};
    const int i = i0 + li, j = j0 + li;
    // the lane's row of op(A) and column of op(B) (clamped to a valid one and masked),
    // walked in steps of 4 along k, in batches of kU steps whose loads are all issued
    // before any of them is used; the last, partial batch is masked the same way (no
    // serial tail of dependent loads)
    constexpr int kU = 8;
    const bool iok = i < M, jok = j < N;
    const long sa = ta ? 1 : lda, sb = tb ? ldb : 1;
    const R* pa = (ta ? A + (long)(iok ? i : 0) * lda : A + (iok ? i : 0)) + lk * sa;
    const R* pb = (tb ? B + (jok ? j : 0) : B + (long)(jok ? j : 0) * ldb) + lk * sb;
    int k0 = 0;
    for (; k0 + 4 * kU <= K; k0 += 4 * kU) {
        R a[kU], b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            a[u] = pa[(long)(4 * u) * sa];
            b[u] = pb[(long)(4 * u) * sb];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) acc = Mma<R>::op(iok ? a[u] : (R)0, jok ? b[u] : (R)0, acc);
        pa += (long)(4 * kU) * sa;
        pb += (long)(4 * kU) * sb;
    }
    if (k0 < K) {
        const int rem = K - k0 - lk;   // this lane's steps left: u < rem / 4 (rounded up)
        R a[kU], b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const bool ok = 4 * u < rem;
            a[u] = (ok && iok) ? pa[(long)(4 * u) * sa] : (R)0;
            b[u] = (ok && jok) ? pb[(long)(4 * u) * sb] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (4 * u < K - k0) acc = Mma<R>::op(a[u], b[u], acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ii = i0 + Mma<R>::row(v, lane), jj = j0 + li;
        if (ii < M && jj < N) {
            const long o = ii + (long)jj * ldc;
            C[o] = (beta == (R)0 ? (R)0 : beta * Cin[o]) + alpha * acc[v];
        }
    }
}

// C (M x N, column-major, ldc) = beta C + alpha op(A) op(B), op(A) M x K, op(B) K x N;
// ta/tb select the transposes (A[k + i*lda] / B[j + k*ldb]).  All threads of the
// workgroup call it; 16 x 16 output tiles are spread over the waves.  With
// upper != 0 tiles entirely below the diagonal are skipped (symmetric results
// whose upper triangle is used).  NW: waves of the workgroup.  Ends with a workgroup
// barrier.
template <typename R, int NW = kWaves>
__device__ void wg_gemm(int M, int N, int K, R alpha, const R* A, int lda, bool ta, const R* B, int ldb,
                        bool tb, R beta, R* C, int ldc, bool upper = false) {
    const int wid = threadIdx.x >> 6;
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
    for (int t = wid; t < tm * tn; t += NW) {
        const int i0 = (t % tm) << 4, j0 = (t / tm) << 4;
        if (upper && i0 > j0 + 15) continue;
        tile_gemm<R>(i0, j0, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, C, ldc);
    }
    __syncthreads();
}

// The same product with bfloat16 operands (rounded to nearest even) and FP32
// accumulation, on v_mfma_f32_16x16x16bf16_1k: A[i][k] in lane i + 16 (k/4),
// element k%4; B[k][j] in lane j + 16 (k/4), element k%4; accumulator as f32.
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
    unsigned u = __float_as_uint(x);
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
    return (short)u;
}

__device__ __forceinline__ void tile_gemm_bf16(int i0, int j0, int M, int N, int K, float alpha, const float* A,
                                               int lda, bool ta, const float* B, int ldb, bool tb, float beta,
                                               const float* Cin, float* C, int ldc) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    v4 acc = {0, 0, 0, 0};
    const int i = i0 + li, j = j0 + li;
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int kk = k0 + 4 * lk + e;
            float va = 0.f, vb = 0.f;
            if (i < M && kk < K) va = ta ? A[kk + (long)i * lda] : A[i + (long)kk * lda];
            if (j < N && kk < K) vb = tb ? B[j + (long)kk * ldb] : B[kk + (long)j * ldb];
            a[e] = bf16_bits(va);
            b[e] = bf16_bits(vb);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int ii = i0 + 4 * lk + v, jj = j0 + li;
        if (ii < M && jj < N) {
            const long o = ii + (long)jj * ldc;
            C[o] = (beta == 0.f ? 0.f : beta * Cin[o]) + alpha * acc[v];
        }
    }
}

template <int NW = kWaves>
__device__ void wg_gemm_bf16(int M, int N, int K, float alpha, const float* A, int lda, bool ta, const float* B,
                             int ldb, bool tb, float beta, float* C, int ldc, bool upper = false) {
    const int wid = threadIdx.x >> 6;
    const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
    for (int t = wid; t < tm * tn; t += NW) {
        const int i0 = (t % tm) << 4, j0 = (t / tm) << 4;
        if (upper && i0 > j0 + 15) continue;
        tile_gemm_bf16(i0, j0, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, C, ldc);
    }
    __syncthreads();
}

// Schur-complement products of the elimination: FP64/FP32 MFMA, or bfloat16
// operands with FP32 accumulation when BF16 is set (float storage only).
template <typename R, bool BF16, int NT = kThreads>
__device__ __forceinline__ void schur_gemm(int M, int N, int K, R alpha, const R* A, int lda, bool ta, const R* B,
                                           int ldb, bool tb, R beta, R* C, int ldc, bool upper = false) {
    if constexpr (BF16)
        wg_gemm_bf16<NT / 64>(M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, upper);
    else
        wg_gemm<R, NT / 64>(M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, upper);
}

// T = R11^{-1} R12 by blocked back substitution over 16-row blocks, bottom up:
// T_I = R_II^{-1} (R12_I - R_{I,>I} T_{>I}); the update is an MFMA GEMM, the
// diagonal solve one column per thread.  All threads of the workgroup call it.
__device__ void id_coefficients(const double* Yb, int m, int np, int k, double* T, int c_lo, int c_hi) {
    __shared__ double s_rblk[16][17];
    __shared__ double s_x[16][kThreads];
    const int nr = c_hi - c_lo;
    if (nr <= 0 || k == 0) return;
    T += (long)c_lo * k;
    for (long e = threadIdx.x; e < (long)k * nr; e += kThreads) {
        const int a = (int)(e % k), c = (int)(e / k);
        T[e] = Yb[a + (long)(k + c_lo + c) * m];
    }
    __syncthreads();
    const int nblk = (k + 15) / 16;
    for (int bi = nblk - 1; bi >= 0; --bi) {
        const int I = bi * 16, ib = min(16, k - I), rest = k - (I + ib);
        if (rest > 0)
            wg_gemm<double>(ib, nr, rest, -1.0, Yb + I + (long)(I + ib) * m, m, false, T + I + ib, k, false, 1.0,
                            T + I, k);
        // the diagonal block of R11 to LDS, and each thread's column of the block to its own
        // LDS lane (s_x[u][thread], conflict-free), so the solve's dependent steps wait on
        // LDS instead of global memory; the same operations in the same order as in place
        for (int e = threadIdx.x; e < ib * ib; e += kThreads) {
            const int a = e % ib, q = e / ib;
            s_rblk[a][q] = Yb[(I + a) + (long)(I + q) * m];
        }
        __syncthreads();
        const int t = threadIdx.x;
        for (int c = t; c < nr; c += kThreads) {
            double* tc = T + (long)c * k + I;
            for (int u = 0; u < ib; ++u) s_x[u][t] = tc[u];
            for (int a = ib - 1; a >= 0; --a) {
                double sum = s_x[a][t];
                for (int q = a + 1; q < ib; ++q) sum -= s_rblk[a][q] * s_x[q][t];
                s_x[a][t] = sum / s_rblk[a][a];
            }
            for (int u = 0; u < ib; ++u) tc[u] = s_x[u][t];
        }
        __syncthreads();
    }
}

constexpr int kBlk = 16;   // block size of the blocked Cholesky / triangular inverse

// Blocked right-looking Cholesky of the upper triangle of S (n x n, lds): S = G^T G,
// G overwrites the upper triangle.  Returns false on a non-positive pivot.
template <typename R, int NT = kThreads>
__device__ bool wg_cholesky_upper(int n, R* S, int lds, int* s_fail) {
    const int tid = threadIdx.x;
    for (int J = 0; J < n; J += kBlk) {
        const int jb = min(kBlk, n - J);
        for (int jj = 0; jj < jb; ++jj) {
            const int c = J + jj;
            if (tid == 0) {
                const R d = S[c + (long)c * lds];
                if (!(d > (R)0)) *s_fail = 1;
                else S[c + (long)c * lds] = sqrt(d);
            }
            __syncthreads();
            if (*s_fail) return false;
            const R g = S[c + (long)c * lds];
            for (int q = c + 1 + tid; q < n; q += NT) S[c + (long)q * lds] /= g;
            __syncthreads();
            // rows c+1 .. J+jb-1 of the block row, all columns right of the diagonal
            const int rows = jb - jj - 1, cols = n - c - 1;
            for (long e = tid; e < (long)rows * cols; e += NT) {
                const int a = c + 1 + (int)(e % rows), q = c + 1 + (int)(e / rows);
                if (q >= a) S[a + (long)q * lds] -= S[c + (long)a * lds] * S[c + (long)q * lds];
            }
            __syncthreads();
        }
        const int rem = n - J - jb;
        if (rem > 0) {
            const R* P = S + J + (long)(J + jb) * lds;   // jb x rem panel of G
            wg_gemm<R, NT / 64>(rem, rem, jb, (R)-1, P, lds, true, P, lds, false, (R)1,
                       S + (J + jb) + (long)(J + jb) * lds, lds, true);
        }
    }
    return true;
}

// X = G^{-1} for upper-triangular G (n x n, ldg), column-block by column-block:
// X_JJ = G_JJ^{-1};  X_{0:J,J} = -X_{0:J,0:J} (G_{0:J,J} X_JJ).  W: n x kBlk scratch.
template <typename R, int NT = kThreads>
__device__ void wg_triangular_inverse(int n, const R* G, int ldg, R* X, R* W) {
    const int tid = threadIdx.x;
    for (long e = tid; e < (long)n * n; e += NT) {
        const int a = (int)(e % n), c = (int)(e / n);
        if (a > c) X[e] = (R)0;
    }
    for (int J = 0; J < n; J += kBlk) {
        const int jb = min(kBlk, n - J);
        for (int c = J + tid; c < J + jb; c += NT) {
            X[c + (long)c * n] = (R)1 / G[c + (long)c * ldg];
            for (int a = c - 1; a >= J; --a) {
                R s = 0;
                for (int b = a + 1; b <= c; ++b) s += G[a + (long)b * ldg] * X[b + (long)c * n];
                X[a + (long)c * n] = -s / G[a + (long)a * ldg];
            }
        }
        __syncthreads();
        if (J > 0) {
            wg_gemm<R, NT / 64>(J, jb, jb, (R)1, G + (long)J * ldg, ldg, false, X + J + (long)J * n, n, false, (R)0, W, J);
            wg_gemm<R, NT / 64>(J, jb, J, (R)-1, X, n, false, W, J, false, (R)0, X + (long)J * n, n);
        }
    }
}

// ---- compress-then-eliminate -------------------------------------------------
// With the box matrix permuted to (s, r) order:
//   B_sr = A_sr - A_ss T,  B_rr = A_rr - T^T A_sr - B_sr^T T   ((e:al))
//   B_rr = G^T G,  E = B_sr G^{-1},  B_ss = A_ss - E E^T      ((e:alu), (e:b))
// B_rr is formed and factored on its upper triangle (it is symmetric in exact
// arithmetic).  The factor slot (np x np elements) receives [T | E | G^{-1} | B_ss].
// A root box has k = 0: its slot receives G^{-1} of the whole box matrix.
// Scratch per box: np^2 + kBig*np elements at its y offset.
//
// Boxes of moderate size: the whole elimination in one workgroup (k_eliminate).
// Large boxes: the same steps as multi-workgroup launch sequences (k_big_gather,
// k_big_gemm, the blocked Cholesky and inverse).
constexpr int kBig = 64;   // block size of the multi-workgroup Cholesky / inverse

template <typename R>
struct ElimView {
    int k, nr, np;
    R *Ass, *Bsr, *Brr, *W, *T, *E, *Gi, *Bss;
};

template <typename R>
__device__ __forceinline__ ElimView<R> elim_view(const BoxMeta& M, int k, R* Wk, R* F) {
    ElimView<R> v;
    v.k = k;
    v.np = M.np;
    v.nr = M.np - k;
    v.Ass = Wk + M.y;
    v.Bsr = v.Ass + (long)k * k;
    v.Brr = v.Bsr + (long)k * v.nr;
    v.W = v.Brr + (long)v.nr * v.nr;
    v.T = F + M.f;
    v.E = v.T + (long)k * v.nr;
    v.Gi = v.E + (long)k * v.nr;
    v.Bss = v.Gi + (long)v.nr * v.nr;
    return v;
}

// Lds: the Cholesky of B_rr and the inverse run on copies in (dynamic) LDS, B_rr and
// G^{-1} n_r x n_r each plus n_r x kBlk scratch, for boxes with n_r <= nr_cap (the host
// reserves that much; a box needing more writes nothing); otherwise they run on the
// box's scratch and factor slot in global memory, where every step of the column
// loop waits on global loads.
template <typename R, bool BF16, bool Lds, int NT>
__global__ __launch_bounds__(NT) void k_eliminate(const BoxMeta* __restrict__ meta,
                                                        const int* __restrict__ list,
                                                        const int* __restrict__ perm,
                                                        const int* __restrict__ kk,
                                                        const R* __restrict__ App,
                                                        const double* __restrict__ T64,
                                                        R* __restrict__ Wk, R* __restrict__ F,
                                                        int* __restrict__ status, int nr_cap) {
    __shared__ int s_fail;
    extern __shared__ char smem_e[];
    const int b = list ? list[blockIdx.x] : blockIdx.x;
    const BoxMeta M = meta[b];
    const ElimView<R> V = elim_view<R>(M, kk[b], Wk, F);
    const int np = V.np, k = V.k, nr = V.nr;
    const int tid = threadIdx.x;
    if (Lds && nr > nr_cap) return;
    if (Lds) {
        R* sS = reinterpret_cast<R*>(smem_e);   // B_rr, then its Cholesky factor G
        R* sX = sS + (long)nr * nr;             // G^{-1}
        R* sW = sX + (long)nr * nr;             // n_r x kBlk scratch of the inverse
        const int* pv = perm + M.act;
        const R* A = App + M.app;
        for (long e = tid; e < (long)k * nr; e += NT) V.T[e] = (R)T64[M.f + e];
        for (long e = tid; e < (long)k * k; e += NT) {
            const int a = (int)(e % k), c = (int)(e / k);
            V.Ass[e] = A[pv[a] + (long)pv[c] * np];
        }
        for (long e = tid; e < (long)k * nr; e += NT) {
            const int a = (int)(e % k), i = (int)(e / k);
            V.Bsr[e] = A[pv[a] + (long)pv[k + i] * np];
        }
        for (long e = tid; e < (long)nr * nr; e += NT) {
            const int i = (int)(e % nr), c = (int)(e / nr);
            V.Brr[e] = A[pv[k + i] + (long)pv[k + c] * np];
        }
        if (tid == 0) s_fail = 0;
        __syncthreads();
        if (k > 0 && nr > 0) {
            schur_gemm<R, BF16, NT>(nr, nr, k, (R)-1, V.T, k, true, V.Bsr, k, false, (R)1, V.Brr, nr, true);   // - T^T A_sr
            schur_gemm<R, BF16, NT>(k, nr, k, (R)-1, V.Ass, k, false, V.T, k, false, (R)1, V.Bsr, k);          // B_sr
            schur_gemm<R, BF16, NT>(nr, nr, k, (R)-1, V.Bsr, k, true, V.T, k, false, (R)1, V.Brr, nr, true);   // - B_sr^T T
        }
        for (long e = tid; e < (long)nr * nr; e += NT) sS[e] = V.Brr[e];
        __syncthreads();
        if (!wg_cholesky_upper<R, NT>(nr, sS, nr, &s_fail)) {
            if (tid == 0) status[0] = b + 1;
            return;
        }
        wg_triangular_inverse<R, NT>(nr, sS, nr, sX, sW);
        for (long e = tid; e < (long)nr * nr; e += NT) V.Gi[e] = sX[e];
        if (k > 0) {
            schur_gemm<R, BF16, NT>(k, nr, nr, (R)1, V.Bsr, k, false, sX, nr, false, (R)0, V.E, k);   // E = B_sr G^{-1}
            for (long e = tid; e < (long)k * k; e += NT) V.Bss[e] = V.Ass[e];
            __syncthreads();
            schur_gemm<R, BF16, NT>(k, k, nr, (R)-1, V.E, k, false, V.E, k, true, (R)1, V.Bss, k);    // B_ss = A_ss - E E^T
        }
        return;
    }
    {
        const int* pv = perm + M.act;
        const R* A = App + M.app;
        for (long e = tid; e < (long)k * nr; e += NT) V.T[e] = (R)T64[M.f + e];
        for (long e = tid; e < (long)k * k; e += NT) {
            const int a = (int)(e % k), c = (int)(e / k);
            V.Ass[e] = A[pv[a] + (long)pv[c] * np];
        }
        for (long e = tid; e < (long)k * nr; e += NT) {
            const int a = (int)(e % k), i = (int)(e / k);
            V.Bsr[e] = A[pv[a] + (long)pv[k + i] * np];
        }
        for (long e = tid; e < (long)nr * nr; e += NT) {
            const int i = (int)(e % nr), c = (int)(e / nr);
            V.Brr[e] = A[pv[k + i] + (long)pv[k + c] * np];
        }
        if (tid == 0) s_fail = 0;
        __syncthreads();
        if (k > 0 && nr > 0) {
            schur_gemm<R, BF16, NT>(nr, nr, k, (R)-1, V.T, k, true, V.Bsr, k, false, (R)1, V.Brr, nr, true);   // - T^T A_sr
            schur_gemm<R, BF16, NT>(k, nr, k, (R)-1, V.Ass, k, false, V.T, k, false, (R)1, V.Bsr, k);          // B_sr
            schur_gemm<R, BF16, NT>(nr, nr, k, (R)-1, V.Bsr, k, true, V.T, k, false, (R)1, V.Brr, nr, true);   // - B_sr^T T
        }
        if (!wg_cholesky_upper<R, NT>(nr, V.Brr, nr, &s_fail)) {
            if (tid == 0) status[0] = b + 1;
            return;
        }
        wg_triangular_inverse<R, NT>(nr, V.Brr, nr, V.Gi, V.W);
    }
    if (k > 0) {
        schur_gemm<R, BF16, NT>(k, nr, nr, (R)1, V.Bsr, k, false, V.Gi, nr, false, (R)0, V.E, k);     // E = B_sr G^{-1}
        for (long e = tid; e < (long)k * k; e += NT) V.Bss[e] = V.Ass[e];
        __syncthreads();
        schur_gemm<R, BF16, NT>(k, k, nr, (R)-1, V.E, k, false, V.E, k, true, (R)1, V.Bss, k);        // B_ss = A_ss - E E^T
    }
}

// Large boxes (np >= kBigElim): the gathers and Schur products of the elimination as
// multi-workgroup launches.  Every workgroup takes kWaves 16 x 16 output tiles of
// one box's product, with the per-tile arithmetic of the one-workgroup path.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_big_gather(const BoxMeta* __restrict__ meta,
                                                         const int* __restrict__ list,
                                                         const int* __restrict__ perm,
                                                         const int* __restrict__ kk,
                                                         const R* __restrict__ App,
                                                         const double* __restrict__ T64,
                                                         R* __restrict__ Wk, R* __restrict__ F) {
    const int b = list[blockIdx.x];
    const BoxMeta M = meta[b];
    const ElimView<R> V = elim_view<R>(M, kk[b], Wk, F);
    const int np = V.np, k = V.k, nr = V.nr;
    const int* pv = perm + M.act;
    const R* A = App + M.app;
    const long n1 = (long)k * nr, n2 = n1 + (long)k * k, n3 = n2 + (long)k * nr, n4 = n3 + (long)nr * nr;
    for (long e = (long)blockIdx.y * kThreads + threadIdx.x; e < n4; e += (long)gridDim.y * kThreads) {
        if (e < n1) {
            V.T[e] = (R)T64[M.f + e];
        } else if (e < n2) {
            const long q = e - n1;
            const int a = (int)(q % k), c = (int)(q / k);
            V.Ass[q] = A[pv[a] + (long)pv[c] * np];
        } else if (e < n3) {
            const long q = e - n2;
            const int a = (int)(q % k), i = (int)(q / k);
            V.Bsr[q] = A[pv[a] + (long)pv[k + i] * np];
        } else {
            const long q = e - n3;
            const int i = (int)(q % nr), c = (int)(q / nr);
            V.Brr[q] = A[pv[k + i] + (long)pv[k + c] * np];
            if (i > c) V.Gi[q] = (R)0;   // lower triangle of G^{-1}
        }
    }
}

// op 0: B_rr -= T^T A_sr; 1: B_sr = A_sr - A_ss T; 2: B_rr -= B_sr^T T (B_rr: upper
// triangle); 3: E = B_sr G^{-1}; 4: B_ss = A_ss - E E^T.
template <typename R, bool BF16>
__global__ __launch_bounds__(kThreads) void k_big_gemm(const BoxMeta* __restrict__ meta,
                                                       const int* __restrict__ list, const int* __restrict__ kk,
                                                       R* __restrict__ Wk, R* __restrict__ F, int op) {
    const int b = list[blockIdx.x];
    const ElimView<R> V = elim_view<R>(meta[b], kk[b], Wk, F);
    const int k = V.k, nr = V.nr;
    if (k == 0 || (op < 3 && nr == 0)) return;
    int Mm, Nn, Kk, lda, ldb, ldc;
    R alpha, beta;
    const R *A, *B, *Cin;
    R* C;
    bool ta = false, tb = false, upper = false;
    switch (op) {
        case 0: Mm = nr; Nn = nr; Kk = k; alpha = -1; A = V.T; lda = k; ta = true; B = V.Bsr; ldb = k;
                beta = 1; C = V.Brr; Cin = C; ldc = nr; upper = true; break;
        case 1: Mm = k; Nn = nr; Kk = k; alpha = -1; A = V.Ass; lda = k; B = V.T; ldb = k;
                beta = 1; C = V.Bsr; Cin = C; ldc = k; break;
        case 2: Mm = nr; Nn = nr; Kk = k; alpha = -1; A = V.Bsr; lda = k; ta = true; B = V.T; ldb = k;
                beta = 1; C = V.Brr; Cin = C; ldc = nr; upper = true; break;
        case 3: Mm = k; Nn = nr; Kk = nr; alpha = 1; A = V.Bsr; lda = k; B = V.Gi; ldb = nr;
                beta = 0; C = V.E; Cin = C; ldc = k; break;
        default: Mm = k; Nn = k; Kk = nr; alpha = -1; A = V.E; lda = k; B = V.E; ldb = k; tb = true;
                 beta = 1; C = V.Bss; Cin = V.Ass; ldc = k; break;
    }
    if constexpr (BF16) {
        const int tm = (Mm + 15) >> 4, tn = (Nn + 15) >> 4;
        for (int t = (int)blockIdx.y * 16 + (threadIdx.x >> 6); t < min(tm * tn, ((int)blockIdx.y + 1) * 16);
             t += kWaves) {
            const int i0 = (t % tm) << 4, j0 = (t / tm) << 4;
            if (upper && i0 > j0 + 15) continue;
            tile_gemm_bf16(i0, j0, Mm, Nn, Kk, alpha, A, lda, ta, B, ldb, tb, beta, Cin, C, ldc);
        }
    } else {
        // one 64 x 64 tile of C per workgroup
        const int tm = (Mm + 63) >> 6, tn = (Nn + 63) >> 6;
        const int t = (int)blockIdx.y;
        if (t >= tm * tn) return;
        const int i0 = (t % tm) << 6, j0 = (t / tm) << 6;
        if (upper && i0 > j0 + 63) return;
        __shared__ BgShared<R> sh;
        if (ta)
            block_gemm64<R, true, false>(sh, i0, j0, Mm, Nn, Kk, alpha, A, lda, B, ldb, beta, Cin, C, ldc, upper);
        else if (tb)
            block_gemm64<R, false, true>(sh, i0, j0, Mm, Nn, Kk, alpha, A, lda, B, ldb, beta, Cin, C, ldc, upper);
        else
            block_gemm64<R, false, false>(sh, i0, j0, Mm, Nn, Kk, alpha, A, lda, B, ldb, beta, Cin, C, ldc, upper);
    }
}

template <typename R>
void launch_big_schur(int nbig, int np_max, const BoxMeta* meta, const int* list, int phase, const int* perm,
                      const int* k, const R* App, const double* T64, R* Wk, R* F, bool bf16, hipStream_t s) {
    if (nbig == 0) return;
    // 64 x 64 tiles of C (the bfloat16 form: sixteen 16 x 16 tiles per workgroup)
    const int t1 = (np_max + 63) / 64;
    const dim3 grid(nbig, t1 * t1);
    auto gemm = [&](int op) {
        if constexpr (sizeof(R) == 4) {
            if (bf16) {
                CBD_LAUNCH((k_big_gemm<R, true>), grid, dim3(kThreads), 0, s, meta, list, k, Wk, F, op);
                return;
            }
        }
        CBD_LAUNCH((k_big_gemm<R, false>), grid, dim3(kThreads), 0, s, meta, list, k, Wk, F, op);
    };
    if (phase == 1) {
        CBD_LAUNCH((k_big_gather<R>), dim3(nbig, 64), dim3(kThreads), 0, s, meta, list, perm, k, App, T64,
                           Wk, F);
        gemm(0);
        gemm(1);
        gemm(2);
    } else {
        gemm(3);
        gemm(4);
    }
}

// Multi-workgroup blocked Cholesky of B_rr (upper, in place) and G^{-1}, for the
// large boxes in `list`; block column J of width kBig per launch step.
// Diagonal block: Cholesky and inverse in LDS (one workgroup per box); the
// inverse goes to the diagonal block of G^{-1}.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_bchol_diag(const BoxMeta* __restrict__ meta,
                                                         const int* __restrict__ list,
                                                         const int* __restrict__ kk, R* __restrict__ Wk,
                                                         R* __restrict__ F, int J, int* __restrict__ status) {
    __shared__ R sA[kBig][kBig + 1];
    __shared__ R sZ[kBig][kBig + 1];
    __shared__ R sP[kWaves][kBig];
    __shared__ R sInv[kBig];
    static_assert(kWaves == 4, "the partial sums below are four");
    const int b = list[blockIdx.x];
    const ElimView<R> V = elim_view<R>(meta[b], kk[b], Wk, F);
    const int nr = V.nr;
    if (J >= nr) return;
    const int jb = min(kBig, nr - J), tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < jb * jb; e += kThreads) {
        const int a = e % jb, c = e / jb;
        sA[a][c] = V.Brr[(J + a) + (long)(J + c) * nr];
    }
    __syncthreads();
    // Right-looking Cholesky, one barrier per step: step j subtracts a_j a_j^T / d_j from
    // the trailing upper triangle (row a = j + 1 + lane, columns of this wave's class
    // mod 4), and scales row j - 1, which no step reads again; the diagonal keeps d_j
    // until the end.
    for (int j = 0; j < jb; ++j) {
        const R d = sA[j][j];
        if (!(d > (R)0)) {
            if (tid == 0) status[0] = b + 1;
            return;
        }
        if (j > 0) {
            const R rp = sqrt(sA[j - 1][j - 1]);
            for (int c = j + tid; c < jb; c += kThreads) sA[j - 1][c] /= rp;
        }
        const int a = j + 1 + lane;
        if (a < jb) {
            const R ga = sA[j][a] / d;
            int c = j + 1 + w;
            if (c < a) c += (a - c + kWaves - 1) / kWaves * kWaves;
            for (; c < jb; c += kWaves) sA[a][c] -= ga * sA[j][c];
        }
        __syncthreads();
    }
    if (tid < jb) sA[tid][tid] = sqrt(sA[tid][tid]);
    __syncthreads();
    // Z = G_JJ^{-1} (upper triangular) by rows from the bottom: row a from the rows
    // below it, each entry's sum split over the four waves
    if (tid < jb) sInv[tid] = (R)1 / sA[tid][tid];
    for (int e = tid; e < jb * jb; e += kThreads) {
        const int a = e % jb, c = e / jb;
        if (a > c) sZ[a][c] = (R)0;
    }
    __syncthreads();
    for (int a = jb - 1; a >= 0; --a) {
        const int c = lane;
        R part = 0;
        if (c > a && c < jb)
            for (int q = a + 1 + w; q <= c; q += kWaves) part += sA[a][q] * sZ[q][c];
        sP[w][lane] = part;
        __syncthreads();
        if (w == 0 && c >= a && c < jb)
            sZ[a][c] = c == a ? sInv[a] : -sInv[a] * ((sP[0][c] + sP[1][c]) + (sP[2][c] + sP[3][c]));
        __syncthreads();
    }
    for (int e = tid; e < jb * jb; e += kThreads) {
        const int a = e % jb, c = e / jb;
        if (a <= c) V.Brr[(J + a) + (long)(J + c) * nr] = sA[a][c];
        V.Gi[(J + a) + (long)(J + c) * nr] = sZ[a][c];
    }
}

// Panel rows J..J+jb of G right of the block: G_J,c = Z^T A_J,c (Z = G_JJ^{-1}),
// kPanel columns per workgroup (each workgroup reads and writes only its columns).
constexpr int kPanel = 128;

template <typename R>
__global__ __launch_bounds__(kThreads) void k_bchol_panel(const BoxMeta* __restrict__ meta,
                                                          const int* __restrict__ list,
                                                          const int* __restrict__ kk, R* __restrict__ Wk,
                                                          R* __restrict__ F, int J) {
    const int b = list[blockIdx.x];
    const ElimView<R> V = elim_view<R>(meta[b], kk[b], Wk, F);
    const int nr = V.nr;
    if (J >= nr) return;
    const int jb = min(kBig, nr - J);
    const int c0 = J + jb + blockIdx.y * kPanel;
    if (c0 >= nr) return;
    const int nc = min(kPanel, nr - c0);
    R* tmp = V.W + (long)c0 * kBig;   // jb x nc, column-major with ld kBig (columns private to this workgroup)
    wg_gemm<R>(jb, nc, jb, (R)1, V.Gi + J + (long)J * nr, nr, true, V.Brr + J + (long)c0 * nr, nr, false, (R)0,
               tmp, kBig);
    for (int e = threadIdx.x; e < jb * nc; e += kThreads) {
        const int a = e % jb, c = e / jb;
        V.Brr[(J + a) + (long)(c0 + c) * nr] = tmp[a + (long)c * kBig];
    }
}

// Trailing update of the upper triangle: S_{rows,cols} -= G_{J,rows}^T G_{J,cols}, one 64 x 64 tile per workgroup.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_bchol_update(const BoxMeta* __restrict__ meta,
                                                           const int* __restrict__ list,
                                                           const int* __restrict__ kk, R* __restrict__ Wk,
                                                           R* __restrict__ F, int J) {
    const int b = list[blockIdx.x];
    const ElimView<R> V = elim_view<R>(meta[b], kk[b], Wk, F);
    const int nr = V.nr;
    if (J >= nr) return;
    const int jb = min(kBig, nr - J);
    const int base = J + jb, rem = nr - base;
    if (rem <= 0) return;
    const int tiles = (rem + 63) / 64;
    const long t = blockIdx.y;
    if (t >= (long)tiles * (tiles + 1) / 2) return;
    // t -> (ti <= tj): tj = floor((sqrt(8t + 1) - 1) / 2)
    int tj = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long)(tj + 1) * (tj + 2) / 2 <= t) ++tj;
    while ((long)tj * (tj + 1) / 2 > t) --tj;
    const int ti = (int)(t - (long)tj * (tj + 1) / 2);
    const int r0 = base + ti * 64, q0 = base + tj * 64;
    const R* P = V.Brr + J;   // panel rows J.., column c at P + c*nr
    __shared__ BgShared<R> sh;
    R* Ct = V.Brr + r0 + (long)q0 * nr;
    block_gemm64<R, true, false>(sh, 0, 0, min(64, nr - r0), min(64, nr - q0), jb, (R)-1, P + (long)r0 * nr, nr,
                                 P + (long)q0 * nr, nr, (R)1, Ct, Ct, nr, ti == tj);
}

// Inverse, block column J > 0: V = G_{0:J,J} Z_J (into W), then
// X_{rows,J} = -X_{rows,rows0:J} V_{rows0:J}, 64 rows per workgroup.
template <typename R>
__global__ __launch_bounds__(kThreads) void k_binv(const BoxMeta* __restrict__ meta,
                                                   const int* __restrict__ list, const int* __restrict__ kk,
                                                   R* __restrict__ Wk, R* __restrict__ F, int J, int stage) {
    const int b = list[blockIdx.x];
    const ElimView<R> V = elim_view<R>(meta[b], kk[b], Wk, F);
    const int nr = V.nr;
    if (J >= nr) return;
    const int jb = min(kBig, nr - J);
    const int r0 = blockIdx.y * 64;
    if (r0 >= J) return;
    const int rows = min(64, J - r0);
    __shared__ BgShared<R> sh;
    if (stage == 0) {
        block_gemm64<R, false, false>(sh, 0, 0, rows, jb, jb, (R)1, V.Brr + r0 + (long)J * nr, nr,
                                      V.Gi + J + (long)J * nr, nr, (R)0, V.W + r0, V.W + r0, nr, false);
    } else {
        R* Ct = V.Gi + r0 + (long)J * nr;
        block_gemm64<R, false, false>(sh, 0, 0, rows, jb, J - r0, (R)-1, V.Gi + r0 + (long)r0 * nr, nr, V.W + r0,
                                      nr, (R)0, Ct, Ct, nr, false);
    }
}

// threads of the elimination's workgroups on the LDS path when the launch's largest n_r
// passes kElimWide (few workgroups fit a CU there; measured at 512^2: 512 threads faster
// for n_r up to 85 and 120, slower for n_r up to 64)
constexpr int kElimLdsThreads = 512;
constexpr int kElimWide = 64;

// elements of LDS the elimination's Cholesky and inverse take for n_r redundant DOFs
static size_t eliminate_lds(int nr) { return (size_t)(2L * nr * nr + (long)nr * kBlk); }

template <typename R>
void launch_eliminate(int nbox, const BoxMeta* meta, const int* list, const int* perm, const int* k,
                      const R* App, const double* T64, R* Wk, R* F, int* status, bool bf16, int nr_max,
                      hipStream_t s) {
    if (nbox == 0) return;
    // the Cholesky and inverse in LDS when the largest B_rr of the launch fits (above
    // 64 KB a workgroup has a CU to itself)
    const size_t shm = eliminate_lds(nr_max) * sizeof(R);
    constexpr int NL = kElimLdsThreads, NG = kThreads;
    size_t lim = std::min(dyn_lds_limit((const void*)k_eliminate<R, false, true, NL>),
                          dyn_lds_limit((const void*)k_eliminate<R, false, true, NG>));
    if constexpr (sizeof(R) == 4)
        lim = std::min({lim, dyn_lds_limit((const void*)k_eliminate<R, true, true, NL>),
                        dyn_lds_limit((const void*)k_eliminate<R, true, true, NG>)});
    const bool lds = nr_max > 0 && shm <= lim;
    const bool wide = nr_max > kElimWide;
    if constexpr (sizeof(R) == 4) {
        if (bf16) {
            if (lds && wide)
                CBD_LAUNCH((k_eliminate<R, true, true, NL>), dim3(nbox), dim3(NL), shm, s, meta, list, perm, k, App,
                           T64, Wk, F, status, nr_max);
            else if (lds)
                CBD_LAUNCH((k_eliminate<R, true, true, NG>), dim3(nbox), dim3(NG), shm, s, meta, list, perm, k, App,
                           T64, Wk, F, status, nr_max);
            else
                CBD_LAUNCH((k_eliminate<R, true, false, NG>), dim3(nbox), dim3(NG), 0, s, meta, list, perm, k, App,
                           T64, Wk, F, status, 0);
            return;
        }
    }
    if (lds && wide)
        CBD_LAUNCH((k_eliminate<R, false, true, NL>), dim3(nbox), dim3(NL), shm, s, meta, list, perm, k, App, T64, Wk,
                   F, status, nr_max);
    else if (lds)
        CBD_LAUNCH((k_eliminate<R, false, true, NG>), dim3(nbox), dim3(NG), shm, s, meta, list, perm, k, App, T64, Wk,
                   F, status, nr_max);
    else
        CBD_LAUNCH((k_eliminate<R, false, false, NG>), dim3(nbox), dim3(NG), 0, s, meta, list, perm, k, App, T64, Wk,
                   F, status, 0);
}

template <typename R>
void launch_big_cholesky_inverse(int nbig, int nr_max, const BoxMeta* meta, const int* list, const int* k,
                                 R* Wk, R* F, int* status, hipStream_t s) {
    if (nbig == 0) return;
    for (int J = 0; J < nr_max; J += kBig) {
        CBD_LAUNCH((k_bchol_diag<R>), dim3(nbig), dim3(kThreads), 0, s, meta, list, k, Wk, F, J, status);
        const int rem = nr_max - J - kBig;
        if (rem > 0) {
            CBD_LAUNCH((k_bchol_panel<R>), dim3(nbig, (rem + kPanel - 1) / kPanel), dim3(kThreads), 0, s,
                               meta, list, k, Wk, F, J);
            const int tiles = (rem + 63) / 64;
            CBD_LAUNCH((k_bchol_update<R>), dim3(nbig, tiles * (tiles + 1) / 2), dim3(kThreads), 0, s,
                               meta, list, k, Wk, F, J);
        }
    }
    for (int J = kBig; J < nr_max; J += kBig) {
        const int chunks = (J + 63) / 64;
        CBD_LAUNCH((k_binv<R>), dim3(nbig, chunks), dim3(kThreads), 0, s, meta, list, k, Wk, F, J, 0);
        CBD_LAUNCH((k_binv<R>), dim3(nbig, chunks), dim3(kThreads), 0, s, meta, list, k, Wk, F, J, 1);
    }
}

// ---- apply ------------------------------------------------------------------
// v: local vectors of all subdomains, slot-major (v[slot * nrhs + c]).
// Slots outside [s0, s1) are set to zero (the apply of one subdomain's term).
// Gather of the subdomains' local vectors, v[slot * nrhs + c] = r[c * N + g] for every
// slot holding grid point g (zero outside the slot range [s0, s1)), 64 points per
// workgroup: a 64-point x 64-column tile of r is read along points (contiguous in r,
// every entry once) into LDS together with the points' slot lists (the inverse map),
// then each wave writes whole slot rows (lane = right-hand side, contiguous in v).
constexpr int kGT = 64;
constexpr int kGatherSlots = 512;   // slot entries of a tile held in LDS (8 per point)
template <typename R>
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ r, long N, int nrhs,
                                                const int* __restrict__ inv_ptr, const int* __restrict__ inv_slot,
                                                long s0, long s1, R* __restrict__ v) {
    __shared__ R tile[kGT][kGT + 1];
    __shared__ int sp[kGT + 1], ss[kGatherSlots];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const long g0 = (long)blockIdx.x * kGT;
    const int npt = (int)min((long)kGT, N - g0);
    if (t <= npt) sp[t] = inv_ptr[g0 + t];
    __syncthreads();
    const int q0 = sp[0], nq = sp[npt] - q0;
    const bool in_lds = nq <= kGatherSlots;
    if (in_lds)
        for (int q = t; q < nq; q += 256) ss[q] = inv_slot[q0 + q];
    for (int c0 = 0; c0 < nrhs; c0 += kGT) {
        const int ncb = min(kGT, nrhs - c0);
        for (int cc = w; cc < ncb; cc += 4)
            tile[lane][cc] = lane < npt ? (R)r[(long)(c0 + cc) * N + g0 + lane] : (R)0;
        __syncthreads();
        if (lane < ncb)
            for (int pt = w; pt < npt; pt += 4) {
                const R x = tile[pt][lane];
                for (int q = sp[pt]; q < sp[pt + 1]; ++q) {
                    const long slot = in_lds ? ss[q - q0] : inv_slot[q];
                    v[slot * nrhs + c0 + lane] = (slot >= s0 && slot < s1) ? x : (R)0;
                }
            }
        __syncthreads();
    }
}

template <typename R>
void launch_gather(const double* r, long N, int nrhs, const int* inv_ptr, const int* inv_slot, long s0, long s1,
                   R* v, hipStream_t s) {
    if (N == 0 || nrhs == 0) return;
    const long b = (N + kGT - 1) / kGT;
    CBD_LAUNCH((k_gather<R>), dim3((unsigned)b), dim3(256), 0, s, r, N, nrhs, inv_ptr, inv_slot, s0, s1, v);
}

// z[:, g] = sum over the subdomain slots holding point g, in a fixed order (the
// inverse map's), for 64 points per workgroup.  The points' slot lists come to LDS
// first; wave w sums the slot rows (lane = right-hand side, contiguous reads) of its 16
// points pt = w, w + 4, ..., taking the q-th slot of all 16 points in one round, so
// their loads are in flight together; each point's sum still adds its slots in the
// inverse map's order.  The sums go through an LDS tile and are written along points
// (contiguous in z).
template <typename R>
__global__ __launch_bounds__(256) void k_scatter(const R* __restrict__ v, int nrhs, const int* __restrict__ inv_ptr,
                                                 const int* __restrict__ inv_slot, long N, double* __restrict__ z) {
    __shared__ double tile[kGT][kGT + 1];
    __shared__ int sp[kGT + 1], ss[kGatherSlots];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const long g0 = (long)blockIdx.x * kGT;
    const int npt = (int)min((long)kGT, N - g0);
    if (t <= npt) sp[t] = inv_ptr[g0 + t];
    __syncthreads();
    const int q0 = sp[0], nq = sp[npt] - q0;
    const bool in_lds = nq <= kGatherSlots;
    if (in_lds)
        for (int q = t; q < nq; q += 256) ss[q] = inv_slot[q0 + q];
    __syncthreads();
    constexpr int kPer = kGT / 4;   // points per wave
    int mult = 0;                   // most slots of one of this wave's points
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int pt = w + 4 * j;
        if (pt < npt) mult = max(mult, sp[pt + 1] - sp[pt]);
    }
    for (int c0 = 0; c0 < nrhs; c0 += kGT) {
        const int ncb = min(kGT, nrhs - c0);
        double acc[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) acc[j] = 0.0;
        if (lane < ncb)
            for (int e = 0; e < mult; ++e) {
#pragma unroll
                for (int j = 0; j < kPer; ++j) {
                    const int pt = w + 4 * j;
                    if (pt < npt && sp[pt] + e < sp[pt + 1]) {
                        const int q = sp[pt] + e;
                        const long slot = in_lds ? ss[q - q0] : inv_slot[q];
                        acc[j] += (double)v[slot * nrhs + c0 + lane];
                    }
                }
            }
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (w + 4 * j < npt) tile[w + 4 * j][lane] = acc[j];
        __syncthreads();
        for (int idx = t; idx < npt * ncb; idx += 256) {
            const int cc = idx / npt, pt = idx % npt;
            z[(long)(c0 + cc) * N + g0 + pt] = tile[pt][cc];
        }
        __syncthreads();
    }
}

template <typename R>
void launch_scatter(const R* v, int nrhs, const int* inv_ptr, const int* inv_slot, long N, double* z,
                    hipStream_t s) {
    if (N == 0 || nrhs == 0) return;
    const long b = (N + kGT - 1) / kGT;
    CBD_LAUNCH((k_scatter<R>), dim3((unsigned)b), dim3(256), 0, s, v, nrhs, inv_ptr, inv_slot, N, z);
}

// One level of the apply sweep, one workgroup of NT threads per (box, chunk of rc
// columns); NT = 512 or 1024 spreads the product tiles of a box over 8 or 16 waves.
// forward:  t = v_r - T^T v_s;  v_r = G^{-T} t;  v_s -= E v_r
// backward: t = v_r - E^T v_s;  v_r = G^{-1} t;  v_s -= T v_r
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_apply_level(const BoxMeta* __restrict__ meta,
                                                          const int* __restrict__ sr,
                                                          const int* __restrict__ kk,
                                                          const R* __restrict__ F, R* __restrict__ v,
                                                          int nbox, int nrhs, int rc, int forward) {
    extern __shared__ char smem_raw[];
    // Workgroup ids go round-robin over the 8 XCDs, each with its own L2: the column
    // groups of one box take ids 8 apart (same XCD, dispatched together), so all but
    // the first read the box's factor from that L2.
    const int ng = (nrhs + rc - 1) / rc;
    const int xcd = (int)(blockIdx.x % 8), slot = (int)(blockIdx.x / 8);
    const int b = (slot / ng) * 8 + xcd, grp = slot % ng;
    if (b >= nbox) return;
    const BoxMeta M = meta[b];
    const int np = M.np, k = kk[b], nr = np - k;
    const int c0 = grp * rc;
    const int nc = (nrhs - c0) < rc ? (nrhs - c0) : rc;
    const int tid = threadIdx.x;
    R* sv = reinterpret_cast<R*>(smem_raw);   // np x rc, rows s then r
    R* tmp = sv + (long)np * rc;              // nr x rc
    const int* ix = sr + M.act;
    for (long e = tid; e < (long)np * nc; e += NT) {
        const int a = (int)(e / nc), c = (int)(e % nc);
        sv[a * rc + c] = v[(long)ix[a] * nrhs + c0 + c];
    }
    __syncthreads();
    if (nr > 0) {
        // the three products (on matrix cores from 8 right-hand sides on), on the transposed
        // local block (column c of v is row c of the nc x np block sv^T, leading dimension rc):
        //   tmp^T = v_r^T - v_s^T X1,  v_r^T = tmp^T G^{-1} (forward) or tmp^T G^{-T},
        //   v_s^T -= v_r^T X2^T   (G^{-1} is stored with a zero lower triangle)
        const R* T = F + M.f;
        const R* E = T + (long)k * nr;
        const R* Gi = E + (long)k * nr;
        R* vs = sv;
        R* vr = sv + (long)k * rc;
        const R* X1 = forward ? T : E;   // applied first (transposed)
        const R* X2 = forward ? E : T;   // applied last
        if (nc >= 8) {
            for (long e = tid; e < (long)nr * rc; e += NT) tmp[e] = vr[e];
            __syncthreads();
            if (k > 0) wg_gemm<R, NT / 64>(nc, nr, k, (R)-1, vs, rc, false, X1, k, false, (R)1, tmp, rc);
            wg_gemm<R, NT / 64>(nc, nr, nr, (R)1, tmp, rc, false, Gi, nr, !forward, (R)0, vr, rc);
            if (k > 0) wg_gemm<R, NT / 64>(nc, k, nr, (R)-1, vr, rc, false, X2, k, true, (R)1, vs, rc);
        } else {
            // a few right-hand sides: one output entry per thread (16 x 16 matrix-core
            // tiles would be mostly empty)
            for (long e = tid; e < (long)nr * nc; e += NT) {
                const int i = (int)(e / nc), c = (int)(e % nc);
                R sum = vr[i * rc + c];
                for (int a = 0; a < k; ++a) sum -= X1[a + (long)i * k] * vs[a * rc + c];
                tmp[i * rc + c] = sum;
            }
            __syncthreads();
            for (long e = tid; e < (long)nr * nc; e += NT) {
                const int i = (int)(e / nc), c = (int)(e % nc);
                R sum = 0;
                if (forward) {
                    for (int j = 0; j <= i; ++j) sum += Gi[j + (long)i * nr] * tmp[j * rc + c];
                } else {
                    for (int j = i; j < nr; ++j) sum += Gi[i + (long)j * nr] * tmp[j * rc + c];
                }
                vr[i * rc + c] = sum;
            }
            __syncthreads();
            for (long e = tid; e < (long)k * nc; e += NT) {
                const int a = (int)(e / nc), c = (int)(e % nc);
                R sum = vs[a * rc + c];
                for (int i = 0; i < nr; ++i) sum -= X2[a + (long)i * k] * vr[i * rc + c];
                vs[a * rc + c] = sum;
            }
            __syncthreads();
        }
    }
    for (long e = tid; e < (long)np * nc; e += NT) {
        const int a = (int)(e / nc), c = (int)(e % nc);
        v[(long)ix[a] * nrhs + c0 + c] = sv[a * rc + c];
    }
}

template <typename R>
size_t apply_level_lds_limit() {
    return std::min({dyn_lds_limit((const void*)k_apply_level<R, 256>), dyn_lds_limit((const void*)k_apply_level<R, 512>),
                     dyn_lds_limit((const void*)k_apply_level<R, 1024>)});
}

template <typename R>
void launch_apply_level(int nbox, const BoxMeta* meta, const int* sr, const int* k, const R* F, R* v,
                        int nrhs, int np_max, int cols, int threads, bool forward, hipStream_t s) {
    if (nbox == 0) return;
    // columns per workgroup: `cols` when given (a tuned choice; the caller has checked
    // its LDS against apply_level_lds_limit), else 16, fewer so that the local copy fits
    // in 64 KiB of LDS (16 measured best over the whole apply at 512^2 with 64
    // right-hand sides: 1.73 ms per apply against 1.77, 2.04 and 2.18 ms for 32, 64 and 8)
    int rc = cols;
    if (rc <= 0) {
        rc = 16;
        while (rc > 1 && (size_t)2 * np_max * rc * sizeof(R) > 65536) rc >>= 1;
    }
    // (boxes whose one column exceeds 64 KB take more, up to the device's limit; the
    // caller has checked that against apply_level_lds_limit)
    if (rc > nrhs) rc = nrhs;
    size_t shm = (size_t)2 * np_max * rc * sizeof(R);
    const long ng = (nrhs + rc - 1) / rc;
    const long blocks = (nbox + 7) / 8 * 8 * ng;
    // 16 waves for boxes of 256 or more DOFs (few boxes, long products), unless given
    if (threads <= 0) threads = np_max >= 256 ? 1024 : 256;
    if (threads == 1024)
        CBD_LAUNCH((k_apply_level<R, 1024>), dim3((unsigned)blocks), dim3(1024), shm, s, meta, sr, k, F, v, nbox,
                   nrhs, rc, forward ? 1 : 0);
    else if (threads == 512)
        CBD_LAUNCH((k_apply_level<R, 512>), dim3((unsigned)blocks), dim3(512), shm, s, meta, sr, k, F, v, nbox,
                   nrhs, rc, forward ? 1 : 0);
    else
        CBD_LAUNCH((k_apply_level<R, 256>), dim3((unsigned)blocks), dim3(256), shm, s, meta, sr, k, F, v, nbox, nrhs,
                   rc, forward ? 1 : 0);
}

// Root boxes too large for the LDS apply: v_root <- G^{-1} G^{-T} v_root as two
// MFMA GEMMs over 64-row chunks, through box-contiguous buffers (column-major,
// ld np, one region of `ts` elements per box).
template <typename R>
__global__ void k_root_move(const BoxMeta* __restrict__ meta, const int* __restrict__ sr, R* __restrict__ v,
                            int nrhs, R* __restrict__ t, long ts, int to_buffer) {
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const long n = (long)M.np * nrhs;
    for (long e = (long)blockIdx.y * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.y * blockDim.x) {
        const int j = (int)(e % M.np), c = (int)(e / M.np);
        R* vv = v + (long)sr[M.act + j] * nrhs + c;
        R* tt = t + b * ts + j + (long)c * M.np;
        if (to_buffer) *tt = *vv;
        else *vv = *tt;
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_root_trmm(const BoxMeta* __restrict__ meta, const R* __restrict__ F,
                                                        int nrhs, const R* __restrict__ in, R* __restrict__ out,
                                                        long ts, int transpose) {
    const int b = blockIdx.x;
    const BoxMeta M = meta[b];
    const int n = M.np;
    const int r0 = blockIdx.y * 64;
    if (r0 >= n) return;
    const int rows = min(64, n - r0);
    // columns c0.. of the right-hand sides: one 16-wide tile column per workgroup, so a
    // wave has one 16 x 16 tile of the 64-row chunk
    const int c0 = blockIdx.z * 16;
    if (c0 >= nrhs) return;
    const int ncol = min(16, nrhs - c0);
    const R* Gi = F + M.f;
    const R* x = in + b * ts + (long)c0 * n;
    R* y = out + b * ts + (long)c0 * n;
    if (transpose) {   // y_rows = (G^{-1})^T x: entries G^{-1}[j][i], j <= i
        const int K = min(n, r0 + 64);
        wg_gemm<R>(rows, ncol, K, (R)1, Gi + (long)r0 * n, n, true, x, n, false, (R)0, y + r0, n);
    } else {           // y_rows = G^{-1} x: entries G^{-1}[i][j], j >= i
        wg_gemm<R>(rows, ncol, n - r0, (R)1, Gi + r0 + (long)r0 * n, n, false, x + r0, n, false, (R)0, y + r0, n);
    }
}

template <typename R>
void launch_root_apply(int nbox, int np_max, int unused, const BoxMeta* meta, const int* sr, const int* k,
                       const R* F, R* v, int nrhs, R* t1, R* t2, hipStream_t s) {
    (void)unused;
    (void)k;
    if (nbox == 0) return;
    const long ts = (long)np_max * nrhs;
    const int chunks = (np_max + 63) / 64, groups = (nrhs + 15) / 16;
    CBD_LAUNCH((k_root_move<R>), dim3(nbox, 64), dim3(256), 0, s, meta, sr, v, nrhs, t1, ts, 1);
    CBD_LAUNCH((k_root_trmm<R>), dim3(nbox, chunks, groups), dim3(kThreads), 0, s, meta, F, nrhs, t1, t2, ts, 1);
    CBD_LAUNCH((k_root_trmm<R>), dim3(nbox, chunks, groups), dim3(kThreads), 0, s, meta, F, nrhs, t2, t1, ts, 0);
    CBD_LAUNCH((k_root_move<R>), dim3(nbox, 64), dim3(256), 0, s, meta, sr, v, nrhs, t1, ts, 0);
}

// ---- the ID from the Gram matrix -------------------------------------------
// For a proxy matrix Y (m x np) the pivoted Cholesky factorization of G = Y^T Y
// chooses the same columns as the column-pivoted QR of Y: after j steps the
// Schur-complement diagonal d_i of G is the squared norm of column i of Y with its
// projection on the j chosen columns removed, i.e. the squared trailing-block norm
// the QR compares.  The Cholesky factor gives R = L^T of that QR (rows up to sign,
// which T = R11^{-1} R12 does not see), so the ID of (e:id) is the same in exact
// arithmetic.  G comes from one product on FP64 matrix cores; the factorization
// runs in panels of kPcholPanel pivots: within a panel (one workgroup per box) each
// new column of L is formed from G's pivot column and the panel's earlier columns
// (left-looking), then the trailing part of G takes the panel's rank-kPcholPanel
// update on matrix cores (many workgroups per box).  Column p of G, once p is
// chosen at step j, holds column j of L; the updates skip chosen rows and columns.
constexpr int kGramTile = 64;              // output tile of the Gram and update products
constexpr int kGramK = 32;                 // rows of Y staged per pass of the Gram product
constexpr int kGramLd = kGramTile + 1;     // LDS row stride (doubles)

__device__ __forceinline__ void lower_tile(int t, int& ti, int& tj) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
}

// G = Y^T Y (np x np, column-major, at goff[b]) for the lower 64 x 64 tiles; each
// off-diagonal tile is also written to its mirror.  Wave w computes a 32 x 32 part
// (2 x 2 blocks of v_mfma_f64_16x16x4f64); Y is staged 32 rows at a time in LDS,
// the next rows loaded into registers during the products.
__global__ __launch_bounds__(kThreads) void k_gram(const BoxMeta* __restrict__ meta, const double* __restrict__ Y,
                                                   const long* __restrict__ goff, double* __restrict__ G) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ double sI[kGramK * kGramLd], sJ[kGramK * kGramLd];
    const int b = blockIdx.y;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np, nt = (np + kGramTile - 1) / kGramTile;
    if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
    int ti, tj;
    lower_tile(blockIdx.x, ti, tj);
    const int I0 = ti * kGramTile, J0 = tj * kGramTile;
    const double* Yb = Y + M.y;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int wi = (wid >> 1) * 32, wj = (wid & 1) * 32;
    constexpr int kCols = kThreads / kGramK;           // columns per staging pass
    constexpr int kPass = kGramTile / kCols;
    const int sr = tid % kGramK, sc = tid / kGramK;
    double nI[kPass], nJ[kPass];
    auto fetch = [&](int k0) {
        const int r = k0 + sr;
#pragma unroll
        for (int u = 0; u < kPass; ++u) {
            const int ci = I0 + sc + kCols * u, cj = J0 + sc + kCols * u;
            nI[u] = (r < m && ci < np) ? Yb[r + (long)ci * m] : 0.0;
            nJ[u] = (r < m && cj < np) ? Yb[r + (long)cj * m] : 0.0;
        }
    };
    v4 acc[2][2];
#pragma unroll
    for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj) acc[qi][qj] = v4{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < m; k0 += kGramK) {
#pragma unroll
        for (int u = 0; u < kPass; ++u) {
            sI[sr * kGramLd + sc + kCols * u] = nI[u];
            sJ[sr * kGramLd + sc + kCols * u] = nJ[u];
        }
        __syncthreads();
        if (k0 + kGramK < m) fetch(k0 + kGramK);
#pragma unroll
        for (int kk = 0; kk < kGramK; kk += 4) {
            double a[2], bb[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = sI[(kk + lk) * kGramLd + wi + 16 * q + li];
                bb[q] = sJ[(kk + lk) * kGramLd + wj + 16 * q + li];
            }
#pragma unroll
            for (int qi = 0; qi < 2; ++qi)
#pragma unroll
                for (int qj = 0; qj < 2; ++qj)
                    acc[qi][qj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[qi], bb[qj], acc[qi][qj], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator (qi, qj) register v: G row i = I0 + wi + 16 qi + 4 v + lk, column j = J0 + wj + 16 qj + li
    double* Gb = G + goff[b];
#pragma unroll
    for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = I0 + wi + 16 * qi + 4 * v + lk, j = J0 + wj + 16 * qj + li;
                if (i < np && j < np) {
                    Gb[j + (long)i * np] = acc[qi][qj][v];
                    if (ti != tj) Gb[i + (long)j * np] = acc[qi][qj][v];
                }
            }
}

// One panel of at most kPcholPanel pivots per box (one workgroup of NT threads per box,
// from step j0; NT = 128, 256 or 512 by the largest box of the batch, so that small
// boxes' steps synchronize fewer waves).  LDS: d (Schur diagonal), pos (column -> position), pv (position -> column).
// Row i of every column of L is read and written by thread i % NT only,
// so the panel's columns need no cross-thread visibility of global memory.  A step
// takes three barriers: the largest remaining norm (each thread's part comes from
// its rows of the previous step's update), the lowest position within the tie
// window (reduced as position * 4096 + column, so the pivot column needs no
// lookup), and the pivot row of the panel's earlier columns.
constexpr int kPcholMaxCols = 16384;  // key range of the pivot reduction (LDS: 16 bytes per column)
template <int NT>
__global__ __launch_bounds__(NT) void k_pchol_panel(const BoxMeta* __restrict__ meta,
                                                               const long* __restrict__ goff, double* __restrict__ G,
                                                               GramState st, int j0, double tol, double tie) {
    extern __shared__ char smem_raw[];
    __shared__ double red[(NT / 64)];
    __shared__ int redi[(NT / 64)];
    __shared__ double s_c[kPcholPanel];
    __shared__ int s_piv[kPcholPanel];
    __shared__ double s_r;
    const int b = blockIdx.x;
    if (j0 > 0 && st.done[b]) return;
    const BoxMeta M = meta[b];
    const int np = M.np, kmax = min(M.m, np);
    double* Gb = G + goff[b];
    double* d = reinterpret_cast<double*>(smem_raw);
    int* pos = reinterpret_cast<int*>(d + np);
    int* pv = pos + np;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    double lm = 0.0;   // largest d over this thread's unchosen rows
    for (int i = tid; i < np; i += NT) {
        const int q = j0 == 0 ? i : st.pos[M.act + i];
        pos[i] = q;
        pv[i] = j0 == 0 ? i : st.pv[M.act + i];
        d[i] = q >= j0 ? Gb[i + (long)i * np] : 0.0;
        if (q >= j0) lm = fmax(lm, d[i]);
    }
    double nu0 = j0 == 0 ? 0.0 : st.nu0[b];
    __syncthreads();
    int taken = 0, stop_k = -1;
    for (int jj = 0; jj < kPcholPanel; ++jj) {
        const int j = j0 + jj;
        if (j >= kmax) {
            stop_k = kmax;
            break;
        }
        lm = wave_max(lm);
        if (lane == 0) red[wid] = lm;
        __syncthreads();
        double mx = red[0];
#pragma unroll
        for (int w = 1; w < (NT / 64); ++w) mx = fmax(mx, red[w]);
        const double nmax = sqrt(mx);
        if (j == 0) nu0 = nmax;
        if (nu0 == 0.0 || nmax <= tol * nu0) {
            stop_k = j;
            break;
        }
        const double thr = nmax - tie * nu0;
        int key = INT_MAX;
        for (int i = tid; i < np; i += NT)
            if (pos[i] >= j && sqrt(fmax(d[i], 0.0)) >= thr) key = min(key, pos[i] * kPcholMaxCols + i);
        key = wave_min_int(key);
        if (lane == 0) redi[wid] = key;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < (NT / 64); ++w) key = min(key, redi[w]);
        const int P = key / kPcholMaxCols, p = key % kPcholMaxCols;
        if (tid == 0) {
            const int q = pv[j];
            pv[j] = p;
            pv[P] = q;
            pos[q] = P;
            pos[p] = j;
            s_piv[jj] = p;
        }
        // row p of the panel's earlier columns, read by the thread that wrote them
        if (tid == p % NT) {
            for (int q = 0; q < jj; ++q) s_c[q] = Gb[p + (long)s_piv[q] * np];
            s_r = sqrt(d[p]);
            st.rdiag[M.act + j] = s_r;
        }
        __syncthreads();
        const double r = s_r;
        double* gp = Gb + (long)p * np;
        lm = 0.0;
        for (int i = tid; i < np; i += NT) {
            if (pos[i] <= j) continue;   // chosen (p now sits at position j)
            double w0 = gp[i], w1 = 0.0, w2 = 0.0, w3 = 0.0;
            int q = 0;
            for (; q + 4 <= jj; q += 4) {
                w0 -= Gb[i + (long)s_piv[q] * np] * s_c[q];
                w1 -= Gb[i + (long)s_piv[q + 1] * np] * s_c[q + 1];
                w2 -= Gb[i + (long)s_piv[q + 2] * np] * s_c[q + 2];
                w3 -= Gb[i + (long)s_piv[q + 3] * np] * s_c[q + 3];
            }
            for (; q < jj; ++q) w0 -= Gb[i + (long)s_piv[q] * np] * s_c[q];
            const double l = ((w0 + w1) + (w2 + w3)) / r;
            gp[i] = l;
            d[i] -= l * l;
            lm = fmax(lm, d[i]);
        }
        taken = jj + 1;
    }
    __syncthreads();
    for (int i = tid; i < np; i += NT) {
        st.pos[M.act + i] = pos[i];
        st.pv[M.act + i] = pv[i];
    }
    if (tid < taken) st.piv[(long)b * kPcholPanel + tid] = s_piv[tid];
    if (tid == 0) {
        st.jend[b] = j0 + taken;
        if (j0 == 0) st.nu0[b] = nu0;
        st.done[b] = stop_k >= 0;
        if (stop_k >= 0) st.k[b] = stop_k;
    }
}

// Trailing update of a panel: G(i, l) -= sum_q L(i, q) L(l, q) over the panel's
// columns q, for rows and columns not yet chosen, in 64 x 64 tiles (all np^2 of
// them) on FP64 MFMA.  The accumulator's lanes run along rows i (consecutive in
// memory): the block computed is L_J L_I^T, whose (l, i) entry updates G(i, l).
__global__ __launch_bounds__(kThreads) void k_pchol_update(const BoxMeta* __restrict__ meta,
                                                           const long* __restrict__ goff, double* __restrict__ G,
                                                           GramState st, int j0) {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __shared__ double sI[kPcholPanel * kGramTile], sJ[kPcholPanel * kGramTile];
    __shared__ int fI[kGramTile], fJ[kGramTile];
    const int b = blockIdx.y;
    const int kt = st.jend[b] - j0;
    // a box that stopped in this panel needs no trailing update: only its chosen columns
    // (L) are read again
    if (kt <= 0 || st.done[b]) return;
    const BoxMeta M = meta[b];
    const int np = M.np, nt = (np + kGramTile - 1) / kGramTile;
    if ((int)blockIdx.x >= nt * nt) return;
    const int I0 = ((int)blockIdx.x % nt) * kGramTile, J0 = ((int)blockIdx.x / nt) * kGramTile;
    const int jend = j0 + kt;
    double* Gb = G + goff[b];
    const int* piv = st.piv + (long)b * kPcholPanel;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, li = lane & 15, lk = lane >> 4;
    for (int e = tid; e < kPcholPanel * kGramTile; e += kThreads) {
        const int q = e / kGramTile, i = e % kGramTile;
        const bool ok = q < kt;
        const long col = ok ? (long)piv[q] * np : 0;
        sI[e] = (ok && I0 + i < np) ? Gb[I0 + i + col] : 0.0;
        sJ[e] = (ok && J0 + i < np) ? Gb[J0 + i + col] : 0.0;
    }
    for (int e = tid; e < kGramTile; e += kThreads) {
        fI[e] = I0 + e < np && st.pos[M.act + I0 + e] >= jend;
        fJ[e] = J0 + e < np && st.pos[M.act + J0 + e] >= jend;
    }
    __syncthreads();
    const int wi = (wid & 1) * 32, wj = (wid >> 1) * 32;
    v4 acc[2][2];
#pragma unroll
    for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj) acc[qi][qj] = v4{0.0, 0.0, 0.0, 0.0};
    const int ksteps = (kt + 3) / 4;
    for (int ks = 0; ks < ksteps; ++ks) {
        const int q = 4 * ks + lk;
        double a[2], bb[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            a[u] = sJ[q * kGramTile + wj + 16 * u + li];    // A(l, q) = L(J0 + l, q)
            bb[u] = sI[q * kGramTile + wi + 16 * u + li];   // B(q, i) = L(I0 + i, q)
        }
#pragma unroll
        for (int qi = 0; qi < 2; ++qi)
#pragma unroll
            for (int qj = 0; qj < 2; ++qj)
                acc[qi][qj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[qj], bb[qi], acc[qi][qj], 0, 0, 0);
    }
    // accumulator (qi, qj) register v: l = wj + 16 qj + 4 v + lk, i = wi + 16 qi + li
#pragma unroll
    for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = wi + 16 * qi + li, l = wj + 16 * qj + 4 * v + lk;
                if (fI[i] && fJ[l]) {
                    double* g = Gb + (I0 + i) + (long)(J0 + l) * np;
                    *g -= acc[qi][qj][v];
                }
            }
}

// R rows 0..k-1 into Y (ld m, columns in position order) as the QR leaves them, and
// k, perm and sr as k_qr_finish writes them.  Workgroup (t, b) takes the 64 x 64 tile t
// of box b's R: row a of R at column c is L(pv[c], a), stored in G's column pv[a], so
// the tile is read along c (rows of one column of G) into LDS and written along a
// (down the columns of Y).  Tile 0 also writes k, perm and sr.
__global__ __launch_bounds__(kThreads) void k_pchol_finish(const BoxMeta* __restrict__ meta,
                                                           const long* __restrict__ goff,
                                                           const double* __restrict__ G, GramState st,
                                                           double* __restrict__ Y, const int* __restrict__ act,
                                                           int* __restrict__ sr, int* __restrict__ perm,
                                                           int* __restrict__ kout) {
    __shared__ double tile[64][65];
    const int b = blockIdx.y;
    const BoxMeta M = meta[b];
    const int m = M.m, np = M.np;
    const int k = st.done[b] ? st.k[b] : min(m, np);
    const int* pv = st.pv + M.act;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        if (tid == 0) kout[b] = k;
        for (int c = tid; c < np; c += kThreads) {
            const int p = pv[c];
            perm[M.act + c] = p;
            sr[M.act + c] = act[M.act + p];
        }
    }
    const int nta = (k + 63) / 64, ntc = (np + 63) / 64;
    if ((int)blockIdx.x >= nta * ntc) return;
    const int a0 = (int)(blockIdx.x % nta) * 64, c0 = (int)(blockIdx.x / nta) * 64;
    const double* Gb = G + goff[b];
    double* Yb = Y + M.y;
    for (int idx = tid; idx < 64 * 64; idx += kThreads) {
        const int cc = idx & 63, aa = idx >> 6, a = a0 + aa, c = c0 + cc;
        double v = 0.0;
        if (a < k && c < np) {
            if (c == a)
                v = st.rdiag[M.act + a];
            else if (c > a)
                v = Gb[pv[c] + (long)pv[a] * np];
        }
        tile[aa][cc] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < 64 * 64; idx += kThreads) {
        const int aa = idx & 63, cc = idx >> 6, a = a0 + aa, c = c0 + cc;
        if (a < k && c < np) Yb[a + (long)c * m] = tile[aa][cc];
    }
}

void launch_gram(int nbox, int np_max, const BoxMeta* meta, const double* Y, const long* goff, double* G,
                 hipStream_t s) {
    if (nbox == 0 || np_max == 0) return;
    const int nt = (np_max + kGramTile - 1) / kGramTile;
    CBD_LAUNCH(k_gram, dim3(nt * (nt + 1) / 2, nbox), dim3(kThreads), 0, s, meta, Y, goff, G);
}
size_t pchol_panel_lds(int np_max) { return (size_t)np_max * (sizeof(double) + 2 * sizeof(int)); }

// Largest dynamic LDS the panel kernel may take on the current device.
size_t pchol_panel_lds_limit() {
    return std::min({dyn_lds_limit((const void*)k_pchol_panel<128>), dyn_lds_limit((const void*)k_pchol_panel<256>),
                     dyn_lds_limit((const void*)k_pchol_panel<512>), pchol_panel_lds(kPcholMaxCols)});
}
void launch_pchol_panel(int nbox, int np_max, const BoxMeta* meta, const long* goff, double* G,
                        const GramState& st, int j0, double tol, double tie, hipStream_t s) {
    if (nbox == 0) return;
    const size_t shm = pchol_panel_lds(np_max);
    if (np_max <= 128)
        CBD_LAUNCH(k_pchol_panel<128>, dim3(nbox), dim3(128), shm, s, meta, goff, G, st, j0, tol, tie);
    else if (np_max <= 256)
        CBD_LAUNCH(k_pchol_panel<256>, dim3(nbox), dim3(256), shm, s, meta, goff, G, st, j0, tol, tie);
    else
        CBD_LAUNCH(k_pchol_panel<512>, dim3(nbox), dim3(512), shm, s, meta, goff, G, st, j0, tol, tie);
    const int nt = (np_max + kGramTile - 1) / kGramTile;
    if (nt > 0) CBD_LAUNCH(k_pchol_update, dim3(nt * nt, nbox), dim3(kThreads), 0, s, meta, goff, G, st, j0);
}
void launch_pchol_finish(int nbox, int np_max, const BoxMeta* meta, const long* goff, const double* G,
                         const GramState& st, double* Y, const int* act, int* sr, int* perm, int* k, double* T64,
                         hipStream_t s) {
    if (nbox == 0) return;
    // 64 x 64 tiles of R (k <= n_p), at least one workgroup per box
    const int nt = (np_max + 63) / 64;
    CBD_LAUNCH(k_pchol_finish, dim3(std::max(1, nt * nt), nbox), dim3(kThreads), 0, s, meta, goff, G, st, Y, act, sr,
               perm, k);
    if (np_max > 0)
        CBD_LAUNCH(k_qr_coeff, dim3(nbox, (np_max + kCoeffCols - 1) / kCoeffCols), dim3(kThreads), 0, s, meta, Y, k,
                   T64);
}

// explicit instantiations
template void launch_proxy_matrix<double>(const ProblemView&, int, const BoxMeta*, const int*,
                                          const int*, const int*, const double*, int, double*,
                                          hipStream_t);
#define CBD_INST(R)                                                                                 \
    template void launch_box_matrix<R>(const ProblemView&, int, int, const BoxMeta*, const int*,    \
                                       const int*, const ChildRef<R>*, R*, hipStream_t);            \
    template void launch_eliminate<R>(int, const BoxMeta*, const int*, const int*, const int*, \
                                      const R*, const double*, R*, R*, int*, bool, int, hipStream_t); \
    template void launch_big_schur<R>(int, int, const BoxMeta*, const int*, int, const int*, const int*, \
                                      const R*, const double*, R*, R*, bool, hipStream_t);          \
    template void launch_big_cholesky_inverse<R>(int, int, const BoxMeta*, const int*, const int*, R*, \
                                                 R*, int*, hipStream_t);                            \
    template void launch_root_apply<R>(int, int, int, const BoxMeta*, const int*, const int*, const R*, \
                                       R*, int, R*, R*, hipStream_t);                               \
    template void launch_gather<R>(const double*, long, int, const int*, const int*, long, long, R*,      \
                                   hipStream_t);                                                    \
    template void launch_scatter<R>(const R*, int, const int*, const int*, long, double*,          \
                                    hipStream_t);                                                   \
    template void launch_apply_level<R>(int, const BoxMeta*, const int*, const int*, const R*, R*,  \
                                        int, int, int, int, bool, hipStream_t);                     \
    template size_t apply_level_lds_limit<R>();
CBD_INST(double)
CBD_INST(float)
#undef CBD_INST

}  // namespace cbd
