// Internal declarations shared by the host runtime (host.cpp) and the HIP
// kernels (*.hip) of libcbd.  Not part of the public ABI (include/cbd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cbd {

// Kernel launches issued by this host thread (the factorization reports its count).
extern thread_local long g_launches;
#define CBD_LAUNCH(...)                \
    do {                               \
        ++::cbd::g_launches;           \
        hipLaunchKernelGGL(__VA_ARGS__); \
    } while (0)

constexpr double kInv2Pi = 0.15915494309189533577;   // 1/(2 pi)
constexpr double kInv4Pi = 0.07957747154594766788;   // 1/(4 pi)

// Read-only view of a discretized problem, passed to kernels by value.
struct ProblemView {
    int d;
    int n;
    long N;
    const double* pts;   // SoA: pts[t*N + g]
    const double* diag;  // b_i c_i A_ii
    const double* w;     // h^d c_j (column scale)
    const double* rs;    // b_i (row scale)
    double spacing;      // distance between neighbouring grid points
};

// Natural logarithm of a positive, finite, normal double.  Range reduction
// x = m 2^e with m in [sqrt(1/2), sqrt(2)), then log m = 2 atanh(s) with
// s = (m - 1)/(m + 1), |s| <= 0.1716, summed as the Taylor series of atanh up
// to s^21 (truncation < 1e-17 relative); e ln 2 uses a two-term split of ln 2
// whose leading term has 25 significant bits, so e * ln2_hi is exact.  The
// quotient uses the hardware reciprocal refined by Newton steps.  Accuracy is
// a few ulp, checked through the matvec against the oracle's libm.
__device__ __forceinline__ double log_pos(double x) {
    constexpr double kLn2Hi = 0x1.62e42fp-1;
    constexpr double kLn2Lo = 0x1.df473de6af279p-26;
    constexpr double kSqrtHalf = 0.70710678118654752440;
    double m = __builtin_amdgcn_frexp_mant(x);          // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool lo = m < kSqrtHalf;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;                            // exact
    const double t = m + 1.0;
    double r = __builtin_amdgcn_rcp(t);
    r = fma(fma(-t, r, 1.0), r, r);
    r = fma(fma(-t, r, 1.0), r, r);
    double s = f * r;
    s = fma(fma(-s, t, f), r, s);                        // s = f / t to ~0.5 ulp
    const double z = s * s;
    double q = 1.0 / 21.0;
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    const double s2 = s + s;
    const double logm = fma(s2 * z, q, s2);              // 2s (1 + z/3 + z^2/5 + ...)
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, logm));
}

// Laplace kernel value K(r) from r^2 (Section 2.1, (e:k)).
template <int D>
__device__ __forceinline__ double laplace_from_r2(double r2) {
    if constexpr (D == 2) {
        return -0.5 * kInv2Pi * log_pos(r2);    // -(1/2pi) log r = -(1/4pi) log r^2
    } else {
        return kInv4Pi * rsqrt(r2);             // 1/(4 pi r)
    }
}

// Entry A_bc[gi][gj] of the discretized operator, generated on the fly in FP64.
template <int D>
__device__ __forceinline__ double matrix_entry(const ProblemView& P, long gi, long gj) {
    if (gi == gj) return P.diag[gi];
    double r2 = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        double dx = P.pts[t * P.N + gi] - P.pts[t * P.N + gj];
        r2 += dx * dx;
    }
    return P.rs[gi] * laplace_from_r2<D>(r2) * P.w[gj];
}

// One box of a level batch of the RS factorization.
struct BoxMeta {
    int sub;        // subdomain
    int np;         // active DOFs of the box (columns of its ID)
    int nnear;      // near-field rows of its proxy matrix
    int m;          // rows of the proxy matrix = nnear + n_pxy (0 for a root box)
    long act;       // offset of its slot lists (act, sr, perm) in the level arrays
    long near;      // offset of its near-field list
    long y;         // offset of its proxy-matrix / elimination scratch (elements)
    long app;       // offset of its box matrix A_pp (np x np, elements)
    long f;         // offset of its factor slot (np x np elements) in the level's factor array
    long ch;        // offset of its child-info entries, -1 for a box made of grid points
    double ctr[3];  // proxy centre
    double rho;     // proxy radius
};

// Where an active DOF of a parent box sits in its child's B_ss.
template <typename R>
struct ChildRef {
    const R* bss;   // child's B_ss (k_c x k_c, column-major)
    int ldk;        // k_c
    int pos;        // position of the DOF among the child's skeletons
};

// ---- launchers (defined in the .hip files) --------------------------------

void launch_assemble(int d, int n, int grid, const double* b, const double* c, double* pts,
                     double* diag, double* w, double* rs, double a_self, double weight,
                     hipStream_t s);
// rb: row blocks of 16 per wave (0: default); max_blocks > 0 limits the grid to the
// first rows (used by the tile autotuner).
void launch_matvec(const ProblemView& P, int nrhs, const double* x, double* y, int rb, int max_blocks,
                   hipStream_t s);
int matvec_rows_per_block(int rb);
int matvec_nb(int nrhs);
bool matvec_prepare();   // per-device constant tables of the matvec (call outside stream capture)
int matvec_default_rb(int nb);

template <typename R>
void launch_proxy_matrix(const ProblemView& P, int nbox, const BoxMeta* meta, const int* act,
                         const int* nearl, const int* cidx, const double* pxdir, int npxy,
                         R* Y, hipStream_t s);
void launch_cpqr(int nbox, const BoxMeta* meta, double* Y, const int* act, int* sr, int* perm,
                 int* k, double* T64, double tol, double tie, int m_max, int np_max, hipStream_t s);

// State of the stepped pivoted QR between launches (per-level device arrays).
// Register-resident pivoted QR of small boxes (at most 256 rows and 104 columns): one
// 512-thread workgroup per box; outputs as launch_cpqr.
bool cpqr_reg_fits(int m_max, int np_max);
void launch_cpqr_reg(int nbox, int np_max, int m_max, const BoxMeta* meta, double* Y, const int* act, int* sr,
                     int* perm, int* k, double* T64, double tol, double tie, hipStream_t s);
struct QrState {
    double* norms;   // remaining column norms, per box at its act offset
    double* alpha;   // diagonal of R, per box at its act offset
    int* pv;         // column order, per box at its act offset
    double* beta;    // per box: 2 / ||v||^2 of the current reflector
    double* nu0;     // per box: largest column norm of Y
    int* done;       // per box: stopped
    int* k;          // per box: rank once stopped
};
// ID by pivoted Cholesky of the Gram matrix (rs.hip): state between panel launches.
constexpr int kPcholPanel = 32;   // pivots per panel
struct GramState {
    double* rdiag;   // R_jj, per box at its act offset (by step)
    int* pv;         // position -> column, per box at its act offset
    int* pos;        // column -> position, per box at its act offset
    int* piv;        // per box: the columns chosen in the current panel (kPcholPanel)
    double* nu0;     // per box: largest column norm of Y
    int* done;       // per box: stopped
    int* k;          // per box: rank once stopped
    int* jend;       // per box: steps taken so far
};
void launch_gram(int nbox, int np_max, const BoxMeta* meta, const double* Y, const long* goff, double* G,
                 hipStream_t s);
size_t pchol_panel_lds(int np_max);
size_t pchol_panel_lds_limit();
size_t dyn_lds_limit(const void* kernel);
template <typename R>
size_t apply_level_lds_limit();
void launch_pchol_panel(int nbox, int np_max, const BoxMeta* meta, const long* goff, double* G,
                        const GramState& st, int j0, double tol, double tie, hipStream_t s);
void launch_pchol_finish(int nbox, int np_max, const BoxMeta* meta, const long* goff, const double* G,
                         const GramState& st, double* Y, const int* act, int* sr, int* perm, int* k, double* T64,
                         hipStream_t s);
void launch_qr_init(int nbox, int np_max, const BoxMeta* meta, const double* Y, const QrState& st,
                    hipStream_t s);
void launch_qr_step(int nbox, int np_max, int m_max, const BoxMeta* meta, double* Y, const QrState& st,
                    int j, double tol, double tie, hipStream_t s);
void launch_qr_finish(int nbox, int np_max, const BoxMeta* meta, double* Y, const QrState& st, const int* act,
                      int* sr, int* perm, int* k, double* T64, hipStream_t s);
// Randomized ID: Z = Omega Y for every box with zmeta[b].m = ell > 0 (Z at zmeta[b].y,
// ell x np column-major); keys: one box key per box.
void launch_sketch(int nbox, int np_max, long mw_max, const BoxMeta* meta, const BoxMeta* zmeta, const double* Y,
                   const int* nearl, const int* cidx, long N, unsigned long long seed,
                   const unsigned long long* keys, const long* boff, unsigned* bits, double* Z, hipStream_t s);
// Row compression before the stepped pivoted QR: Householder QR of every box's Y
// (meta), then R (min(m, np) x np) into Rc at the offsets of cmeta.  Tw: nbox x
// kHqrTw doubles; alpha: one double per active DOF (meta's act offsets); Vbuf:
// nbox x kHqrVbuf(m_max) doubles of reflector staging.
constexpr int kHqrTw = 32 * 32;
inline long kHqrVbuf(int m_max) { return 2L * m_max * 32; }
void launch_hqr(int nbox, int np_max, int m_max, int k_max, const BoxMeta* meta, double* Y, double* Tw,
                double* alpha, double* Vbuf, const BoxMeta* cmeta, double* Rc, hipStream_t s);
template <typename R>
void launch_box_matrix(const ProblemView& P, int nbox, int np_max, const BoxMeta* meta, const int* act,
                       const int* cidx, const ChildRef<R>* ch, R* App, hipStream_t s);
// the whole elimination of each box in one workgroup (list: box indices or NULL)
// bf16: Schur-complement products with bfloat16 operands and FP32 accumulation (R = float)
template <typename R>
void launch_eliminate(int nbox, const BoxMeta* meta, const int* list, const int* perm,
                      const int* k, const R* App, const double* T64, R* Wk, R* F, int* status,
                      bool bf16, int nr_max, hipStream_t s);
// the elimination of the boxes in list as multi-workgroup launches: phase 1 up to B_rr,
// phase 2 E and B_ss (the arithmetic of launch_eliminate, spread over many workgroups)
template <typename R>
void launch_big_schur(int nbig, int np_max, const BoxMeta* meta, const int* list, int phase, const int* perm,
                      const int* k, const R* App, const double* T64, R* Wk, R* F, bool bf16, hipStream_t s);
// multi-workgroup blocked Cholesky of B_rr and G^{-1} for the boxes in list (after phase 1)
template <typename R>
void launch_big_cholesky_inverse(int nbig, int nr_max, const BoxMeta* meta, const int* list, const int* k,
                                 R* Wk, R* F, int* status, hipStream_t s);
// v_root <- G^{-1} G^{-T} v_root for every (k = 0) box of a root level, via buffers t1, t2
// of nbox * np_max * nrhs elements each
template <typename R>
void launch_root_apply(int nbox, int np_max, int unused, const BoxMeta* meta, const int* sr, const int* k,
                       const R* F, R* v, int nrhs, R* t1, R* t2, hipStream_t s);
constexpr int kBigBox = 512;        // roots with at least this many DOFs are applied by GEMMs
constexpr int kBigElim = 256;       // boxes with at least this many DOFs are eliminated by the
                                    // multi-workgroup path (512^2 factor 23 -> 21.5 ms against 512)
constexpr int kScratchCols = 64;    // elimination scratch per box: np^2 + kScratchCols * np

// v[slot * nrhs + c] = r[c * N + g] for the slots in [s0, s1) holding grid point g (the
// inverse map inv_ptr/inv_slot), zero for the other slots
template <typename R>
void launch_gather(const double* r, long N, int nrhs, const int* inv_ptr, const int* inv_slot, long s0, long s1,
                   R* v, hipStream_t s);
template <typename R>
void launch_scatter(const R* v, int nrhs, const int* inv_ptr, const int* inv_slot, long N,
                    double* z, hipStream_t s);
template <typename R>
void launch_apply_level(int nbox, const BoxMeta* meta, const int* sr, const int* k, const R* F,
                        R* v, int nrhs, int np_max, int cols, int threads, bool forward, hipStream_t s);

// Matvec by FFT (fft.hip): ghat (P^d reals) is the transform of the kernel's circulant
// generator; tw[k] = exp(-2 pi i k / P), k < P/2; buf holds max_pairs complex P^d arrays.
void launch_fft_prepare(const ProblemView& Pv, int P, int logP, double spacing, double2* gbuf, double* ghat,
                        const double2* tw, hipStream_t s);
void launch_matvec_fft(const ProblemView& Pv, int P, int logP, const double* ghat, const double2* tw,
                       double2* buf, int max_pairs, int nrhs, const double* x, double* y, hipStream_t s);

// PCG vector kernels (FP64).
void launch_dot(const double* a, const double* b, long N, int nrhs, double* partial,
                double* out, hipStream_t s);
void launch_pcg_alpha(const double* rz, const double* pq, const int* active, double* alpha,
                      int nrhs, hipStream_t s);
void launch_pcg_update_ur(double* u, double* r, const double* p, const double* q,
                          const double* alpha, long N, int nrhs, hipStream_t s);
void launch_pcg_beta(const double* rz_new, double* rz, const int* active, double* beta,
                     int nrhs, hipStream_t s);
void launch_pcg_update_p(double* p, const double* z, const double* beta, long N, int nrhs,
                         hipStream_t s);
void launch_copy(double* dst, const double* src, long n, hipStream_t s);
void launch_fill(double* dst, double v, long n, hipStream_t s);
void launch_sub(double* dst, const double* a, const double* b, long n, hipStream_t s);
// 4-byte words (bytes a multiple of 4): copy; flag = 1 where a differs from ref; *p = v
void launch_copy_words(void* dst, const void* src, size_t bytes, hipStream_t s);
void launch_check_words(const void* a, const void* ref, size_t bytes, int* flag, hipStream_t s);
void launch_set_word(int* p, int v, hipStream_t s);

constexpr int kDotBlocks = 256;   // partial sums per right-hand side in launch_dot

// Skeleton-rank predictor (mlp.hip).
constexpr int kMlpFeatures = 6;
constexpr int kMlpWidth = 64;
constexpr int kMlpParams = kMlpWidth * kMlpFeatures + kMlpWidth + kMlpWidth * kMlpWidth + kMlpWidth +
                           kMlpWidth + 1;
void launch_mlp_forward(const float* p, int n, const float* X, float* y, float* z1, float* z2,
                        hipStream_t s);
// ws: (2 + 4 * kMlpWidth) * n floats
void launch_mlp_loss_grad(const float* p, int n, const float* X, const float* t, float* grad,
                          float* loss, float* ws, hipStream_t s);
void launch_mlp_adam(float* p, const float* g, float* m, float* v, int step, float lr, hipStream_t s);
// Samples the library-owned loss/gradient scratch holds (rank_mlp_loss_grad_noalloc),
// and its device address on the current device (nullptr if it cannot be had).
constexpr int kMlpStaticMax = 16384;
float* mlp_static_scratch();

}  // namespace cbd
