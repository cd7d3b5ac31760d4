// Host runtime of libcbd: the C ABI of include/cbd.h, the domain decomposition
// and box hierarchy (Sections 2.2-2.3, 3.2), the level-batched RS factorization
// driver, the preconditioner apply and the PCG loop (Section 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cbd.h"
#include "internal.h"

using namespace cbd;

// ---------------------------------------------------------------------------
// errors, timing
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                           \
    do {                                                                                    \
        hipError_t e_ = (x);                                                                \
        if (e_ != hipSuccess) return fail(CBD_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char* cbd_last_error(void) { return g_err.c_str(); }

namespace {

std::mutex g_tmx;
bool g_timing = false;
thread_local bool g_capturing = false;   // no timer events inside a stream capture
struct PendingTimer {
    std::string name;
    hipEvent_t a, b;
};
std::vector<PendingTimer> g_pending;
std::map<std::string, std::pair<double, long>> g_acc;

// Records HIP events on `stream` around a launch sequence when timing is on.
struct ScopedTimer {
    std::string name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    ScopedTimer(const char* n, hipStream_t st) : name(n), s(st) {
        std::lock_guard<std::mutex> lk(g_tmx);
        if (!g_timing || g_capturing) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        (void)hipEventRecord(a, s);
        on = true;
    }
    ~ScopedTimer() {
        if (!on) return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_tmx);
        g_pending.push_back({name, a, b});
    }
};

void resolve_timers() {
    std::lock_guard<std::mutex> lk(g_tmx);
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto& acc = g_acc[p.name];
            acc.first += ms;
            acc.second += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}

}  // namespace

extern "C" int cbd_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmx);
    g_timing = on != 0;
    return CBD_OK;
}

extern "C" int cbd_timing_get(const char* name, double* total_ms, long* launches) {
    if (!name) return fail(CBD_EARG, "cbd_timing_get: name is NULL");
    resolve_timers();
    std::lock_guard<std::mutex> lk(g_tmx);
    auto it = g_acc.find(name);
    if (total_ms) *total_ms = it == g_acc.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == g_acc.end() ? 0 : it->second.second;
    return CBD_OK;
}

extern "C" int cbd_timing_reset(void) {
    resolve_timers();
    std::lock_guard<std::mutex> lk(g_tmx);
    g_acc.clear();
    return CBD_OK;
}

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------
struct cbd_problem_s {
    int d, n, grid;
    long N;
    double h, weight, a_self;
    double *pts, *diag, *w, *rs;
    int mv_rb[4] = {0, 0, 0, 0};   // tuned matvec row blocks per wave, per RHS-block count (0: default)
    // FFT matvec state (cbd_fft_prepare)
    int fft_P = 0, fft_logP = 0, fft_pairs = 0;
    double* fft_ghat = nullptr;
    double2* fft_tw = nullptr;
    double2* fft_buf = nullptr;
    ~cbd_problem_s() {
        if (fft_ghat) (void)hipFree(fft_ghat);
        if (fft_tw) (void)hipFree(fft_tw);
        if (fft_buf) (void)hipFree(fft_buf);
    }
    ProblemView view() const { return ProblemView{d, n, N, pts, diag, w, rs}; }
};

// Exact integral of K over the cell [-h/2, h/2]^d (diagonal of (e:a_2d)/(e:a_3d)).
static double self_cell(int d, double h) {
    const double pi = 3.14159265358979323846;
    if (d == 2) return -(h * h / (2.0 * pi)) * (std::log(h) - 0.5 * std::log(2.0) - 1.5 + pi / 4.0);
    return (3.0 * h * h / (4.0 * pi)) * (std::log(2.0 + std::sqrt(3.0)) - pi / 6.0);
}

extern "C" int ie_assemble(int d, int n, int grid, const double* b, const double* c, double* pts,
                           double* diag, double* w, double* rowscale, void* stream,
                           cbd_problem* out) {
    if (!out) return fail(CBD_EARG, "ie_assemble: out is NULL");
    if (d != 2 && d != 3) return fail(CBD_EARG, "ie_assemble: d must be 2 or 3");
    if (n < 2) return fail(CBD_EARG, "ie_assemble: n must be >= 2");
    if (grid != CBD_GRID_CELL && grid != CBD_GRID_NODE) return fail(CBD_EARG, "ie_assemble: bad grid");
    if (grid == CBD_GRID_NODE && d != 2) return fail(CBD_EARG, "ie_assemble: node grid is 2D only");
    if (!pts || !diag || !w || !rowscale) return fail(CBD_EARG, "ie_assemble: output pointer is NULL");
    long N = 1;
    for (int t = 0; t < d; ++t) N *= n;
    if (N > (1L << 30)) return fail(CBD_EARG, "ie_assemble: N too large");
    auto* p = new cbd_problem_s;
    p->d = d;
    p->n = n;
    p->grid = grid;
    p->N = N;
    p->h = 1.0 / n;
    p->weight = std::pow(p->h, d);
    p->a_self = self_cell(d, p->h);
    p->pts = pts;
    p->diag = diag;
    p->w = w;
    p->rs = rowscale;
    hipStream_t s = (hipStream_t)stream;
    if (!matvec_prepare()) {
        delete p;
        return fail(CBD_ENOMEM, "ie_assemble: could not allocate the matvec tables");
    }
    launch_assemble(d, n, grid, b, c, pts, diag, w, rowscale, p->a_self, p->weight, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        delete p;
        return fail(CBD_EHIP, std::string("ie_assemble launch: ") + hipGetErrorString(e));
    }
    *out = p;
    return CBD_OK;
}

extern "C" int cbd_problem_free(cbd_problem p) {
    delete p;
    return CBD_OK;
}

extern "C" int kernel_matvec(cbd_problem p, int nrhs, const double* x, double* y, void* stream) {
    if (!p || !x || !y || nrhs < 1) return fail(CBD_EARG, "kernel_matvec: bad argument");
    if (x == y) return fail(CBD_EARG, "kernel_matvec: x and y alias");
    hipStream_t s = (hipStream_t)stream;
    {
        ScopedTimer tm("matvec", s);
        launch_matvec(p->view(), nrhs, x, y, p->mv_rb[matvec_nb(nrhs) - 1], 0, s);
    }
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int cbd_fft_prepare(cbd_problem p, int max_pairs, void* stream) {
    if (!p || max_pairs < 1) return fail(CBD_EARG, "cbd_fft_prepare: bad argument");
    int P = 2, logP = 1;
    while (P < 2 * p->n - 1) {
        P <<= 1;
        ++logP;
    }
    if (P > 4096) return fail(CBD_EARG, "cbd_fft_prepare: transform length above 4096 (n > 2048)");
    long vol = 1;
    for (int t = 0; t < p->d; ++t) vol *= P;
    hipStream_t s = (hipStream_t)stream;
    if (p->fft_ghat) (void)hipFree(p->fft_ghat);
    if (p->fft_tw) (void)hipFree(p->fft_tw);
    if (p->fft_buf) (void)hipFree(p->fft_buf);
    p->fft_ghat = nullptr;
    p->fft_tw = nullptr;
    p->fft_buf = nullptr;
    p->fft_P = 0;
    HIPCHK(hipMalloc(&p->fft_ghat, sizeof(double) * vol));
    HIPCHK(hipMalloc(&p->fft_tw, sizeof(double2) * (P / 2)));
    HIPCHK(hipMalloc(&p->fft_buf, sizeof(double2) * vol * max_pairs));
    std::vector<double2> tw(P / 2);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < P / 2; ++k) tw[k] = make_double2(std::cos(2.0 * pi * k / P), -std::sin(2.0 * pi * k / P));
    HIPCHK(hipMemcpy(p->fft_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice));
    const double spacing = p->grid == CBD_GRID_CELL ? 1.0 / p->n : 1.0 / (p->n - 1);
    launch_fft_prepare(p->view(), P, logP, spacing, p->fft_buf, p->fft_ghat, p->fft_tw, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    p->fft_P = P;
    p->fft_logP = logP;
    p->fft_pairs = max_pairs;
    return CBD_OK;
}

extern "C" int kernel_matvec_fft(cbd_problem p, int nrhs, const double* x, double* y, void* stream) {
    if (!p || !x || !y || nrhs < 1) return fail(CBD_EARG, "kernel_matvec_fft: bad argument");
    if (x == y) return fail(CBD_EARG, "kernel_matvec_fft: x and y alias");
    if (!p->fft_P) return fail(CBD_EARG, "kernel_matvec_fft: call cbd_fft_prepare first");
    hipStream_t s = (hipStream_t)stream;
    {
        ScopedTimer tm("matvec_fft", s);
        launch_matvec_fft(p->view(), p->fft_P, p->fft_logP, p->fft_ghat, p->fft_tw, p->fft_buf, p->fft_pairs, nrhs,
                          x, y, s);
    }
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int cbd_autotune_matvec(cbd_problem p, int nrhs, void* stream, int* choice) {
    if (!p || nrhs < 1) return fail(CBD_EARG, "cbd_autotune_matvec: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = matvec_nb(nrhs);
    const int cols = std::min(nrhs, 64);
    double *x = nullptr, *y = nullptr;
    HIPCHK(hipMalloc(&x, sizeof(double) * p->N * cols));
    HIPCHK(hipMalloc(&y, sizeof(double) * p->N * cols));
    launch_fill(x, 1.0, p->N * cols, s);
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int best = matvec_default_rb(nb);
    double best_t = 1e300;
    const int cand[3] = {1, 2, 4};
    for (int rb : cand) {
        // every candidate runs on the same number of workgroups (4 per CU when the
        // grid is that large), so that occupancy and L2 reuse are comparable
        const long rows = matvec_rows_per_block(rb);
        const long full = (p->N + rows - 1) / rows;
        const int blocks = (int)std::min(full, 1024L);
        launch_matvec(p->view(), cols, x, y, rb, blocks, s);   // warm-up
        (void)hipEventRecord(a, s);
        for (int rep = 0; rep < 2; ++rep) launch_matvec(p->view(), cols, x, y, rb, blocks, s);
        (void)hipEventRecord(b, s);
        float ms = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) continue;
        const double per_row = ms / (double)(blocks * rows);
        if (per_row < best_t) {
            best_t = per_row;
            best = rb;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(x);
    (void)hipFree(y);
    HIPCHK(hipGetLastError());
    p->mv_rb[nb - 1] = best;
    if (choice) *choice = best;
    return CBD_OK;
}

// ---------------------------------------------------------------------------
// partition and box hierarchy
// ---------------------------------------------------------------------------
namespace {

struct Leaf {
    int lo[3], hi[3];
    int start, count;
};
struct PBox {
    int lo[3], hi[3];
    std::vector<int> children;
    int parent = -1;
    int first_leaf = 0;
};
struct Sub {
    std::vector<int> index;                 // global indices in local order
    std::vector<Leaf> leaves;
    std::vector<std::vector<PBox>> levels;  // levels[l] boxes
    int root_level = 0;
    long offset = 0;                        // first slot of this subdomain
};

int ceil_log2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

struct cbd_partition_s {
    int d, n, m, delta, mode, leaf_side, Lt, Lr;
    std::vector<Sub> subs;
    long total = 0;
    // device copies, uploaded on first use
    int* d_cidx = nullptr;      // slot -> global index
    int* d_inv_ptr = nullptr;   // N+1
    int* d_inv_slot = nullptr;  // total
    std::vector<int> cidx;
    int upload() {
        if (d_cidx) return CBD_OK;
        long N = 1;
        for (int t = 0; t < d; ++t) N *= n;
        std::vector<int> cnt(N + 1, 0);
        for (long e = 0; e < total; ++e) cnt[cidx[e] + 1]++;
        for (long g = 0; g < N; ++g) cnt[g + 1] += cnt[g];
        std::vector<int> slot(total), fill(cnt.begin(), cnt.end() - 1);
        for (long e = 0; e < total; ++e) slot[fill[cidx[e]]++] = (int)e;
        HIPCHK(hipMalloc(&d_cidx, sizeof(int) * total));
        HIPCHK(hipMalloc(&d_inv_ptr, sizeof(int) * (N + 1)));
        HIPCHK(hipMalloc(&d_inv_slot, sizeof(int) * total));
        HIPCHK(hipMemcpy(d_cidx, cidx.data(), sizeof(int) * total, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_inv_ptr, cnt.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_inv_slot, slot.data(), sizeof(int) * total, hipMemcpyHostToDevice));
        return CBD_OK;
    }
    ~cbd_partition_s() {
        if (d_cidx) (void)hipFree(d_cidx);
        if (d_inv_ptr) (void)hipFree(d_inv_ptr);
        if (d_inv_slot) (void)hipFree(d_inv_slot);
    }
};

extern "C" int dd_partition(int d, int n, int m, int delta, int mode, int leaf_side,
                            cbd_partition* out) {
    if (!out) return fail(CBD_EARG, "dd_partition: NULL argument");
    if (d != 2 && d != 3) return fail(CBD_EARG, "dd_partition: d must be 2 or 3");
    if (n < 2) return fail(CBD_EARG, "dd_partition: n must be >= 2");
    if (m < 1 || n % m != 0) return fail(CBD_EARG, "dd_partition: n must be a multiple of m");
    if (delta < 0 || leaf_side < 0) return fail(CBD_EARG, "dd_partition: negative delta or leaf_side");
    if (mode != CBD_MODE_JACOBI && mode != CBD_MODE_SCHWARZ && mode != CBD_MODE_CBD)
        return fail(CBD_EARG, "dd_partition: unknown mode");
    if (mode == CBD_MODE_JACOBI) delta = 0;
    const int s = n / m;
    if (mode == CBD_MODE_CBD && m > 2 && 2 * delta > s)
        return fail(CBD_EARG, "dd_partition: CBD needs 2*delta <= n/m");

    struct Region {
        int kp[3], lo[3], hi[3];
    };
    int M = 1;
    for (int t = 0; t < d; ++t) M *= m;
    const int D = (mode == CBD_MODE_CBD) ? (1 << d) : M;
    std::vector<std::vector<Region>> regs(D);
    for (int kl = 0; kl < M; ++kl) {
        int k[3] = {0, 0, 0}, r = kl;
        for (int t = 0; t < d; ++t) {
            k[t] = r % m;
            r /= m;
        }
        Region g{};
        for (int t = 0; t < d; ++t) {
            g.lo[t] = std::max(0, k[t] * s - delta);
            g.hi[t] = std::min(n, (k[t] + 1) * s + delta);
            g.kp[t] = (mode == CBD_MODE_CBD) ? k[t] / 2 : 0;
        }
        int target = kl;
        if (mode == CBD_MODE_CBD) {
            target = 0;
            for (int t = 0; t < d; ++t) target += (k[t] % 2) << t;
        }
        regs[target].push_back(g);
    }
    auto tiles = [&](const int* lo, const int* hi, int* T) {
        for (int t = 0; t < d; ++t)
            T[t] = leaf_side <= 0 ? 1 : (hi[t] - lo[t] + leaf_side - 1) / leaf_side;
    };
    int qmax = 1, rmax = 1;
    for (auto& rl : regs)
        for (auto& g : rl) {
            int T[3];
            tiles(g.lo, g.hi, T);
            for (int t = 0; t < d; ++t) {
                qmax = std::max(qmax, T[t]);
                rmax = std::max(rmax, g.kp[t] + 1);
            }
        }
    auto* q = new cbd_partition_s;
    q->d = d;
    q->n = n;
    q->m = m;
    q->delta = delta;
    q->mode = mode;
    q->leaf_side = leaf_side;
    q->Lt = ceil_log2(qmax);
    q->Lr = ceil_log2(rmax);
    q->subs.resize(D);
    long offset = 0;
    for (int i = 0; i < D; ++i) {
        Sub& sd = q->subs[i];
        sd.offset = offset;
        std::vector<std::array<int, 6>> leaf_key;   // kp[3], q[3]
        for (auto& g : regs[i]) {
            int T[3] = {1, 1, 1};
            tiles(g.lo, g.hi, T);
            int nt = 1;
            for (int t = 0; t < d; ++t) nt *= T[t];
            for (int ql = 0; ql < nt; ++ql) {
                int qq[3] = {0, 0, 0}, r = ql;
                for (int t = 0; t < d; ++t) {
                    qq[t] = r % T[t];
                    r /= T[t];
                }
                Leaf lf{};
                for (int t = 0; t < d; ++t) {
                    if (leaf_side <= 0) {
                        lf.lo[t] = g.lo[t];
                        lf.hi[t] = g.hi[t];
                    } else {
                        lf.lo[t] = g.lo[t] + qq[t] * leaf_side;
                        lf.hi[t] = std::min(g.hi[t], g.lo[t] + (qq[t] + 1) * leaf_side);
                    }
                }
                lf.start = (int)sd.index.size();
                // points of the tile, x fastest
                int ext[3] = {1, 1, 1};
                for (int t = 0; t < d; ++t) ext[t] = lf.hi[t] - lf.lo[t];
                for (int c2 = 0; c2 < (d == 3 ? ext[2] : 1); ++c2)
                    for (int c1 = 0; c1 < ext[1]; ++c1)
                        for (int c0 = 0; c0 < ext[0]; ++c0) {
                            long g0 = lf.lo[0] + c0, g1 = lf.lo[1] + c1, g2 = d == 3 ? lf.lo[2] + c2 : 0;
                            sd.index.push_back((int)(g0 + (long)n * g1 + (long)n * n * g2));
                        }
                lf.count = (int)sd.index.size() - lf.start;
                sd.leaves.push_back(lf);
                std::array<int, 6> key{};
                for (int t = 0; t < d; ++t) {
                    key[t] = g.kp[t];
                    key[3 + t] = qq[t];
                }
                leaf_key.push_back(key);
            }
        }
        offset += (long)sd.index.size();
        // levels: a leaf's key at level l decides its box; boxes in order of first appearance
        std::vector<int> leaf_box_prev;
        for (int l = 0;; ++l) {
            std::map<std::array<int, 6>, int> where;
            std::vector<PBox> boxes;
            std::vector<int> leaf_box(sd.leaves.size());
            const int sr_ = std::max(0, l - q->Lt), sq_ = std::min(l, q->Lt);
            for (size_t li = 0; li < sd.leaves.size(); ++li) {
                std::array<int, 6> key{};
                for (int t = 0; t < d; ++t) {
                    key[t] = leaf_key[li][t] >> sr_;
                    key[3 + t] = leaf_key[li][3 + t] >> sq_;
                }
                auto it = where.find(key);
                int bi;
                if (it == where.end()) {
                    bi = (int)boxes.size();
                    where[key] = bi;
                    PBox b;
                    for (int t = 0; t < 3; ++t) {
                        b.lo[t] = sd.leaves[li].lo[t];
                        b.hi[t] = sd.leaves[li].hi[t];
                    }
                    b.first_leaf = (int)li;
                    boxes.push_back(b);
                } else {
                    bi = it->second;
                }
                PBox& b = boxes[bi];
                for (int t = 0; t < d; ++t) {
                    b.lo[t] = std::min(b.lo[t], sd.leaves[li].lo[t]);
                    b.hi[t] = std::max(b.hi[t], sd.leaves[li].hi[t]);
                }
                leaf_box[li] = bi;
            }
            if (l > 0) {
                auto& prev = sd.levels[l - 1];
                for (size_t c = 0; c < prev.size(); ++c) {
                    int pb = leaf_box[prev[c].first_leaf];
                    boxes[pb].children.push_back((int)c);
                    prev[c].parent = pb;
                }
            }
            sd.levels.push_back(std::move(boxes));
            leaf_box_prev = leaf_box;
            if (sd.levels.back().size() == 1) {
                sd.root_level = l;
                break;
            }
        }
    }
    q->total = offset;
    q->cidx.resize(offset);
    for (auto& sd : q->subs)
        for (size_t e = 0; e < sd.index.size(); ++e) q->cidx[sd.offset + e] = sd.index[e];
    *out = q;
    return CBD_OK;
}

extern "C" int cbd_partition_free(cbd_partition q) {
    delete q;
    return CBD_OK;
}

extern "C" int dd_partition_info(cbd_partition q, int* D, int* Lt, int* Lr, long* total) {
    if (!q) return fail(CBD_EARG, "dd_partition_info: NULL partition");
    if (D) *D = (int)q->subs.size();
    if (Lt) *Lt = q->Lt;
    if (Lr) *Lr = q->Lr;
    if (total) *total = q->total;
    return CBD_OK;
}

extern "C" int dd_subdomain_info(cbd_partition q, int i, int* size, int* n_leaves, int* root_level) {
    if (!q || i < 0 || i >= (int)q->subs.size()) return fail(CBD_EARG, "dd_subdomain_info: bad index");
    const Sub& sd = q->subs[i];
    if (size) *size = (int)sd.index.size();
    if (n_leaves) *n_leaves = (int)sd.leaves.size();
    if (root_level) *root_level = sd.root_level;
    return CBD_OK;
}

extern "C" int dd_subdomain_index(cbd_partition q, int i, int* index) {
    if (!q || !index || i < 0 || i >= (int)q->subs.size()) return fail(CBD_EARG, "dd_subdomain_index: bad argument");
    std::memcpy(index, q->subs[i].index.data(), sizeof(int) * q->subs[i].index.size());
    return CBD_OK;
}

extern "C" int dd_level_boxes(cbd_partition q, int i, int level, int* n_boxes, int* lohi, int* parent) {
    if (!q || i < 0 || i >= (int)q->subs.size()) return fail(CBD_EARG, "dd_level_boxes: bad subdomain");
    const Sub& sd = q->subs[i];
    if (level < 0 || level > sd.root_level) return fail(CBD_EARG, "dd_level_boxes: bad level");
    const auto& bx = sd.levels[level];
    if (n_boxes) *n_boxes = (int)bx.size();
    for (size_t b = 0; b < bx.size(); ++b) {
        if (lohi)
            for (int t = 0; t < q->d; ++t) {
                lohi[b * 2 * q->d + t] = bx[b].lo[t];
                lohi[b * 2 * q->d + q->d + t] = bx[b].hi[t];
            }
        if (parent) parent[b] = bx[b].parent;
    }
    return CBD_OK;
}

// ---------------------------------------------------------------------------
// factor
// ---------------------------------------------------------------------------
namespace {

template <typename T>
T* dalloc(size_t n, int& rc) {
    T* p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, sizeof(T) * n) != hipSuccess) {
        rc = fail(CBD_ENOMEM, "hipMalloc failed");
        return nullptr;
    }
    return p;
}

struct Level {
    bool root = false;
    int nbox = 0;
    std::vector<BoxMeta> meta;
    std::vector<int> k, sr;             // host copies after the level ran
    std::vector<int> box_sub, box_idx;  // subdomain and partition box index of each batch box
    std::vector<int> side;              // box side in cells (proxy geometry)
    std::vector<int> sub_start;         // first batch index of each subdomain (-1: absent)
    int np_max = 0, m_max = 0;
    long tot_act = 0, tot_f = 0;
    BoxMeta* d_meta = nullptr;
    int *d_act = nullptr, *d_sr = nullptr, *d_perm = nullptr, *d_k = nullptr;
    void* d_F = nullptr;
    void release() {
        if (d_meta) (void)hipFree(d_meta);
        if (d_act) (void)hipFree(d_act);
        if (d_sr) (void)hipFree(d_sr);
        if (d_perm) (void)hipFree(d_perm);
        if (d_k) (void)hipFree(d_k);
        if (d_F) (void)hipFree(d_F);
        d_meta = nullptr;
        d_act = d_sr = d_perm = d_k = nullptr;
        d_F = nullptr;
    }
};

// grow-only device buffer
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t b) {
        if (b <= bytes) return CBD_OK;
        if (p) {
            // queued kernels of an earlier level may still use the old buffer
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, b) != hipSuccess) return fail(CBD_ENOMEM, "hipMalloc of workspace failed");
        bytes = b;
        return CBD_OK;
    }
    ~DevBuf() {
        if (p) {
            (void)hipDeviceSynchronize();
            (void)hipFree(p);
        }
    }
};

}  // namespace

struct cbd_factor_s {
    cbd_problem_s* prob;
    cbd_partition_s* part;
    int prec;
    double tol = 0.0;
    // scheduling statistics of the factorization
    int host_syncs = 0;       // stream synchronizations issued by the factorization
    int qr_steps = 0;         // launch pairs of the stepped pivoted QR
    int mispredicted = 0;     // stepped boxes whose rank exceeded the predicted step budget
    int hqr_levels = 0;       // stepped batches whose proxy matrices were row-compressed first
    int sketched = 0;         // boxes whose ID came from a sketch
    int sketch_fallbacks = 0; // boxes whose sketch saturated (deterministic ID instead)
    int chunks = 0;           // level chunks (more than the number of levels when the workspace is bounded)
    double pred_abs_err = 0.0;
    int pred_count = 0;
    size_t esize;
    std::vector<Level> levels;   // compressed levels, then the root level
    int n_compress = 0;
    std::vector<int> S;
    size_t bytes = 0;
    double flops = 0.0;
    DevBuf v;                    // local vectors of the apply
    DevBuf t1, t2;               // root-level buffers of the apply for large roots
    ~cbd_factor_s() {
        for (auto& l : levels) l.release();
    }
};

namespace {

// Levels with at least this many boxes run the ID with one workgroup per box;
// fewer boxes use the stepped QR that spreads each box over many workgroups.
constexpr int kStepBoxes = 1024;

// Randomized ID: rows of the sketch of an m x np proxy matrix (0: no sketch), and the
// margin below ell that a sketch's rank must stay under to be accepted.
constexpr int kSketchOver = 8;
int sketch_rows(int m, int np) {
    const int ell = (3 * np + 4) / 5 + kSketchOver;
    return ell < std::min(m, np) ? ell : 0;
}

double cpqr_flops(double m, double n, double k) {
    return 4.0 * m * n * k - 2.0 * (m + n) * k * k + 4.0 * k * k * k / 3.0;
}
double elim_flops(double k, double nr) {
    // T solve, B_sr, B_rr (symmetric), Cholesky, G^{-1}, E, B_ss (symmetric)
    return k * k * nr + 2.0 * k * k * nr + 2.0 * nr * nr * k + nr * nr * nr / 3.0 + nr * nr * nr / 3.0 +
           k * nr * nr + k * k * nr;
}

// Features of a box known before its ID (input of the rank predictor).
void box_features(int level, int side, int np, int nnear, double tol, int d, float* out) {
    out[0] = (float)level / 4.f;
    out[1] = (float)std::log2((double)std::max(side, 1)) / 4.f;
    out[2] = (float)std::log2((double)std::max(np, 1)) / 8.f;
    out[3] = (float)std::log2((double)nnear + 1.0) / 8.f;
    out[4] = (float)(-std::log10(std::max(tol, 1e-300))) / 8.f;
    out[5] = (float)d / 3.f;
}

// Proxy surface directions: equispaced circle (2D), golden-angle sphere (3D).
std::vector<double> proxy_dirs(int d, int npxy) {
    std::vector<double> dir((size_t)npxy * d);
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < npxy; ++j) {
        if (d == 2) {
            double th = 2.0 * pi * j / npxy;
            dir[j * 2] = std::cos(th);
            dir[j * 2 + 1] = std::sin(th);
        } else {
            double z = 1.0 - (2.0 * j + 1.0) / npxy;
            double rr = std::sqrt(1.0 - z * z);
            double phi = j * (pi * (3.0 - std::sqrt(5.0)));
            dir[j * 3] = rr * std::cos(phi);
            dir[j * 3 + 1] = rr * std::sin(phi);
            dir[j * 3 + 2] = z;
        }
    }
    return dir;
}

template <typename R>
int factor_impl(cbd_problem_s* P, cbd_partition_s* Q, const cbd_rs_opts* o, hipStream_t s,
                cbd_factor_s* F) {
    int rc = Q->upload();
    if (rc) return rc;
    const int d = P->d, n = P->n;
    const ProblemView PV = P->view();
    const int D = (int)Q->subs.size();
    const int npxy = o->exact ? 0 : o->n_pxy;
    // The ID (proxy matrix, pivoted QR, T) always runs in FP64: at tol ~ 1e-6 the
    // FP32 round-off floor of the recomputed column norms reaches the tolerance
    // and the ranks inflate.  Elimination, storage and apply use R.
    const double tie = 1e-10;
    const bool bf16 = o->precision == CBD_PREC_BF16GEMM;
    std::vector<double> hdir = proxy_dirs(d, std::max(npxy, 1));
    DevBuf dirbuf, ybuf, wbuf, t64buf, appbuf, nearbuf, chbuf, statbuf, qrbuf, mlpbuf, listbuf, hqrbuf, idbuf, zbuf;
    if ((rc = dirbuf.ensure(sizeof(double) * hdir.size()))) return rc;
    HIPCHK(hipMemcpyAsync(dirbuf.p, hdir.data(), sizeof(double) * hdir.size(), hipMemcpyHostToDevice, s));

    int Lmax = 0;
    if (!o->exact)
        for (auto& sd : Q->subs) Lmax = std::max(Lmax, sd.root_level);
    F->n_compress = Lmax;
    // one Cholesky-breakdown slot per level, read once at the end: the host plans a
    // level while the previous level's elimination runs
    if ((rc = statbuf.ensure(sizeof(int) * (Lmax + 1)))) return rc;
    HIPCHK(hipMemsetAsync(statbuf.p, 0, sizeof(int) * (Lmax + 1), s));
    std::vector<std::vector<int>> keep;   // host sources of uploads still in flight
    // grid coordinates of a global index
    // half-cell coordinates 2 j_t + 1 of every slot (near-field tests in integers)
    const long nslot = (long)Q->cidx.size();
    std::vector<int> hc((size_t)d * nslot);
    for (long e = 0; e < nslot; ++e) {
        int g = Q->cidx[e];
        for (int t = 0; t < d; ++t) {
            hc[(size_t)t * nslot + e] = 2 * (g % n) + 1;
            g /= n;
        }
    }
    const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));

    for (int l = 0; l <= Lmax; ++l) {
        const bool root = (l == Lmax);
        F->levels.emplace_back();
        Level& L = F->levels.back();
        L.root = root;
        L.sub_start.assign(D, -1);
        std::vector<std::vector<int>> act;      // slot lists per batch box
        std::vector<std::vector<ChildRef<R>>> chl;
        std::vector<int> blo, bhi;              // box bounds (3 per box)
        for (int i = 0; i < D; ++i) {
            const Sub& sd = Q->subs[i];
            if (!root && (o->exact || sd.root_level <= l)) continue;
            L.sub_start[i] = L.nbox;
            // which partition level the boxes of this batch come from
            const int pl = root ? (o->exact ? -1 : sd.root_level) : l;
            const int nb = root ? 1 : (int)sd.levels[l].size();
            for (int b = 0; b < nb; ++b) {
                std::vector<int> a;
                std::vector<ChildRef<R>> ch;
                int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
                if (pl < 0) {   // exact: the whole subdomain
                    for (size_t e = 0; e < sd.index.size(); ++e) a.push_back((int)(sd.offset + e));
                } else {
                    const PBox& pb = sd.levels[pl][b];
                    for (int t = 0; t < 3; ++t) {
                        lo[t] = pb.lo[t];
                        hi[t] = pb.hi[t];
                    }
                    if (pl == 0) {
                        const Leaf& lf = sd.leaves[b];
                        a.resize(lf.count);
                        for (int e = 0; e < lf.count; ++e) a[e] = (int)(sd.offset + lf.start + e);
                    } else {
                        const Level& PLv = F->levels[pl - 1];
                        int nsk = 0;
                        for (int c : pb.children) nsk += PLv.k[PLv.sub_start[i] + c];
                        a.reserve(nsk);
                        ch.reserve(nsk);
                        for (int c : pb.children) {
                            const int cb = PLv.sub_start[i] + c;
                            const BoxMeta& cm = PLv.meta[cb];
                            const int kc = PLv.k[cb], nrc = cm.np - kc;
                            const R* bss = (const R*)PLv.d_F + cm.f + 2L * kc * nrc + (long)nrc * nrc;
                            for (int e = 0; e < kc; ++e) {
                                a.push_back(PLv.sr[cm.act + e]);
                                ch.push_back(ChildRef<R>{bss, kc, e});
                            }
                        }
                    }
                }
                act.push_back(std::move(a));
                chl.push_back(std::move(ch));
                for (int t = 0; t < 3; ++t) {
                    blo.push_back(lo[t]);
                    bhi.push_back(hi[t]);
                }
                L.box_sub.push_back(i);
                L.box_idx.push_back(b);
                L.nbox++;
            }
        }
        // near fields (compressed levels only), per subdomain.  Candidate boxes come
        // from a uniform bucket grid over the boxes' lower corners (cell = the
        // largest box side), so the search is linear in the number of boxes.
        std::vector<std::vector<int>> nearl(L.nbox);
        if (!root) {
            struct SubGrid {
                int b0 = -1, nb = 0, smax = 1;
                int glo[3] = {INT_MAX, INT_MAX, INT_MAX}, ghi[3] = {0, 0, 0}, gdim[3] = {1, 1, 1};
                std::vector<std::vector<int>> bucket;
                int cell_of(int t, int x) const { return std::min(gdim[t] - 1, std::max(0, (x - glo[t]) / smax)); }
            };
            std::vector<SubGrid> grids(D);
            for (int i = 0; i < D; ++i) {
                if (L.sub_start[i] < 0) continue;
                SubGrid& G = grids[i];
                G.b0 = L.sub_start[i];
                G.nb = (int)Q->subs[i].levels[l].size();
                for (int b = 0; b < G.nb; ++b)
                    for (int t = 0; t < d; ++t) {
                        G.smax = std::max(G.smax, bhi[(G.b0 + b) * 3 + t] - blo[(G.b0 + b) * 3 + t]);
                        G.glo[t] = std::min(G.glo[t], blo[(G.b0 + b) * 3 + t]);
                        G.ghi[t] = std::max(G.ghi[t], blo[(G.b0 + b) * 3 + t]);
                    }
                for (int t = 0; t < d; ++t) G.gdim[t] = (G.ghi[t] - G.glo[t]) / G.smax + 1;
                G.bucket.resize((size_t)G.gdim[0] * G.gdim[1] * G.gdim[2]);
                for (int b = 0; b < G.nb; ++b) {
                    long ci = 0;
                    for (int t = d - 1; t >= 0; --t) ci = ci * G.gdim[t] + G.cell_of(t, blo[(G.b0 + b) * 3 + t]);
                    G.bucket[ci].push_back(b);
                }
            }
            // the near field of box B (subdomain i, index b): active slots of the other
            // boxes of its subdomain within the proxy radius of its centre
            auto near_of = [&](int B) {
                const SubGrid& G = grids[L.box_sub[B]];
                const int b = B - G.b0;
                int Lside = 0;
                long c2[3] = {0, 0, 0};
                for (int t = 0; t < d; ++t) {
                    Lside = std::max(Lside, bhi[B * 3 + t] - blo[B * 3 + t]);
                    c2[t] = blo[B * 3 + t] + bhi[B * 3 + t];
                }
                const double rad = o->proxy_ratio * Lside;          // grid units
                const double R2 = (2.0 * rad) * (2.0 * rad);        // half-cell units, squared
                int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
                for (int t = 0; t < d; ++t) {
                    // a box reaching within rad of the centre has its lower corner in
                    // [centre - rad - smax, centre + rad]
                    clo[t] = G.cell_of(t, (int)std::floor(0.5 * c2[t] - rad) - G.smax);
                    chi[t] = G.cell_of(t, (int)std::ceil(0.5 * c2[t] + rad));
                }
                std::vector<int> cand;
                cand.reserve(64);
                nearl[B].reserve(8 * act[B].size());
                for (int z = clo[2]; z <= chi[2]; ++z)
                    for (int y = clo[1]; y <= chi[1]; ++y)
                        for (int x = clo[0]; x <= chi[0]; ++x) {
                            const auto& bk = G.bucket[((size_t)z * G.gdim[1] + y) * G.gdim[0] + x];
                            cand.insert(cand.end(), bk.begin(), bk.end());
                        }
                std::sort(cand.begin(), cand.end());   // the order of an all-pairs scan
                for (int b2 : cand) {
                    if (b2 == b) continue;
                    const int B2 = G.b0 + b2;
                    double md = 0.0;
                    for (int t = 0; t < d; ++t) {
                        double lo2 = 2.0 * blo[B2 * 3 + t], hi2 = 2.0 * bhi[B2 * 3 + t];
                        double dd = std::max(0.0, std::max(lo2 - c2[t], c2[t] - hi2));
                        md += dd * dd;
                    }
                    if (md >= R2) continue;
                    for (int slot : act[B2]) {
                        long s2 = 0;
                        for (int t = 0; t < d; ++t) {
                            const long off = hc[(size_t)t * nslot + slot] - c2[t];
                            s2 += off * off;
                        }
                        if ((double)s2 < R2) nearl[B].push_back(slot);
                    }
                }
            };
            // boxes are independent: one pool of host threads over all boxes of the level
            const int nt = std::min(nthreads, std::max(1, L.nbox / 64));
            if (nt <= 1) {
                for (int B = 0; B < L.nbox; ++B) near_of(B);
            } else {
                std::vector<std::thread> pool;
                for (int w = 0; w < nt; ++w)
                    pool.emplace_back([&, w] {
                        for (int B = w; B < L.nbox; B += nt) near_of(B);
                    });
                for (auto& th : pool) th.join();
            }
        }
        // metadata and offsets
        long o_act = 0, o_near = 0, o_y = 0, o_app = 0, o_f = 0, o_ch = 0;
        L.meta.resize(L.nbox);
        for (int B = 0; B < L.nbox; ++B) {
            BoxMeta& M = L.meta[B];
            std::memset(&M, 0, sizeof(M));
            M.sub = L.box_sub[B];
            M.np = (int)act[B].size();
            M.nnear = (int)nearl[B].size();
            M.m = root ? 0 : M.nnear + npxy;
            M.act = o_act;
            M.near = o_near;
            M.y = o_y;
            M.app = o_app;
            M.f = o_f;
            M.ch = chl[B].empty() ? -1 : o_ch;
            int Lside = 0;
            for (int t = 0; t < d; ++t) {
                M.ctr[t] = 0.5 * (blo[B * 3 + t] + bhi[B * 3 + t]) * P->h;
                Lside = std::max(Lside, bhi[B * 3 + t] - blo[B * 3 + t]);
            }
            M.rho = o->proxy_ratio * Lside * P->h;
            L.side.push_back(Lside);
            const long np = M.np;
            o_act += np;
            o_near += M.nnear;
            o_y += std::max((long)M.m * np, np * np + kScratchCols * np);   // proxy matrix, or elimination scratch
            o_app += np * np;
            o_f += np * np;
            o_ch += (long)chl[B].size();
            L.np_max = std::max(L.np_max, M.np);
            L.m_max = std::max(L.m_max, M.m);
        }
        L.tot_act = o_act;
        L.tot_f = o_f;
        // device arrays of the level (kept for the apply)
        L.d_meta = dalloc<BoxMeta>(L.nbox, rc);
        L.d_act = dalloc<int>(o_act, rc);
        L.d_sr = dalloc<int>(o_act, rc);
        L.d_perm = dalloc<int>(o_act, rc);
        L.d_k = dalloc<int>(L.nbox, rc);
        L.d_F = dalloc<R>(o_f, rc);
        if (rc) return rc;
        F->bytes += sizeof(R) * (size_t)o_f;
        // The level's boxes go through the proxy matrices, IDs and elimination in chunks
        // of consecutive boxes whose scratch (Y, elimination work, FP64 T, box matrices)
        // fits the workspace budget; the factor arrays stay level-wide.
        std::vector<int> cut{0};
        long cy = 0, cf = 0, ca = 0, my = 1, mf = 1, ma = 1;
        {
            const double budget = o->workspace_bytes ? (double)o->workspace_bytes : 64.0 * (1L << 30);
            double acc = 0.0;
            for (int B = 0; B < L.nbox; ++B) {
                const BoxMeta& M = L.meta[B];
                const long yb = std::max((long)M.m * M.np, (long)M.np * M.np + kScratchCols * M.np);
                const long fb = (long)M.np * M.np;
                const double bytes = (double)yb * (2 * sizeof(double) + sizeof(R)) + (double)fb * (sizeof(double) + sizeof(R));
                if (B > cut.back() && acc + bytes > budget) {
                    cut.push_back(B);
                    acc = 0.0;
                    cy = cf = ca = 0;
                }
                acc += bytes;
                cy += yb;
                cf += fb;
                ca += fb;
                my = std::max(my, cy);
                mf = std::max(mf, cf);
                ma = std::max(ma, ca);
            }
            cut.push_back(L.nbox);
        }
        F->chunks += (int)cut.size() - 1;
        if ((rc = ybuf.ensure(sizeof(double) * my))) return rc;
        if ((rc = wbuf.ensure(sizeof(R) * my))) return rc;
        if ((rc = t64buf.ensure(sizeof(double) * mf))) return rc;
        if ((rc = appbuf.ensure(sizeof(R) * ma))) return rc;
        if ((rc = nearbuf.ensure(sizeof(int) * std::max(o_near, 1L)))) return rc;
        if ((rc = chbuf.ensure(sizeof(ChildRef<R>) * std::max(o_ch, 1L)))) return rc;
        std::vector<int> hact, hnear;
        std::vector<ChildRef<R>> hch;
        hact.reserve(o_act);
        hnear.reserve(o_near);
        hch.reserve(o_ch);
        for (int B = 0; B < L.nbox; ++B) {
            hact.insert(hact.end(), act[B].begin(), act[B].end());
            hnear.insert(hnear.end(), nearl[B].begin(), nearl[B].end());
            hch.insert(hch.end(), chl[B].begin(), chl[B].end());
        }
        HIPCHK(hipMemcpyAsync(L.d_meta, L.meta.data(), sizeof(BoxMeta) * L.nbox, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(L.d_act, hact.data(), sizeof(int) * o_act, hipMemcpyHostToDevice, s));
        if (o_near)
            HIPCHK(hipMemcpyAsync(nearbuf.p, hnear.data(), sizeof(int) * o_near, hipMemcpyHostToDevice, s));
        if (o_ch)
            HIPCHK(hipMemcpyAsync(chbuf.p, hch.data(), sizeof(ChildRef<R>) * o_ch, hipMemcpyHostToDevice, s));
        R* FF = (R*)L.d_F;
        std::vector<int> kpred;
        std::vector<int> kall, sk_ell;   // ranks (host copy kept for the upload) and sketch rows per box
        if (!root && o->mlp) {
            std::vector<float> feats((size_t)L.nbox * kMlpFeatures), yhat(L.nbox);
            for (int B = 0; B < L.nbox; ++B)
                box_features(l, L.side[B], L.meta[B].np, L.meta[B].nnear, o->tol, d, &feats[(size_t)B * kMlpFeatures]);
            if ((rc = mlpbuf.ensure(sizeof(float) * (size_t)L.nbox * (kMlpFeatures + 1)))) return rc;
            float* dX = (float*)mlpbuf.p;
            float* dy = dX + (size_t)L.nbox * kMlpFeatures;
            HIPCHK(hipMemcpyAsync(dX, feats.data(), sizeof(float) * feats.size(), hipMemcpyHostToDevice, s));
            launch_mlp_forward(o->mlp, L.nbox, dX, dy, nullptr, nullptr, s);
            HIPCHK(hipMemcpyAsync(yhat.data(), dy, sizeof(float) * L.nbox, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            F->host_syncs++;
            kpred.resize(L.nbox);
            for (int B = 0; B < L.nbox; ++B) {
                const int kmax = std::min(L.meta[B].m, L.meta[B].np);
                const double kp = std::exp2((double)yhat[B]) - 1.0;
                kpred[B] = std::max(0, std::min(kmax, (int)std::lround(std::isfinite(kp) ? kp : (double)kmax)));
            }
        }
        kall.assign(L.nbox, 0);
        sk_ell.assign(L.nbox, 0);
        for (size_t ci = 0; ci + 1 < cut.size(); ++ci) {
        const int b0 = cut[ci], b1 = cut[ci + 1], nbc = b1 - b0;
        // chunk-based views: the level's offsets (meta y, f, app) land in the chunk buffers
        double* Y = (double*)ybuf.p - L.meta[b0].y;
        double* T64 = (double*)t64buf.p - L.meta[b0].f;
        R* Wk = (R*)wbuf.p - L.meta[b0].y;
        R* App = (R*)appbuf.p - L.meta[b0].app;
        const BoxMeta* d_meta_c = L.d_meta + b0;
        int* d_k_c = L.d_k + b0;
        int np_max_c = 0;
        for (int B = b0; B < b1; ++B) np_max_c = std::max(np_max_c, L.meta[B].np);
        int* d_status = (int*)statbuf.p + l;
        if (!root) {
            launch_proxy_matrix<double>(PV, nbc, d_meta_c, L.d_act, (const int*)nearbuf.p, Q->d_cidx,
                                        (const double*)dirbuf.p, npxy, Y, s);
            // The ID of a batch of boxes (bm: their metadata, m rows of Ymat each, at the
            // offsets bm[].y), with k into kb (host, one per batch box).
            auto id_batch = [&](const std::vector<BoxMeta>& bm, double* Ymat, const std::vector<int>& bpred,
                                std::vector<int>& kb) -> int {
                const int nb = (int)bm.size();
                kb.assign(nb, 0);
                if (nb == 0) return CBD_OK;
                int m_max = 0, np_max = 0;
                for (const BoxMeta& M : bm) {
                    m_max = std::max(m_max, M.m);
                    np_max = std::max(np_max, M.np);
                }
                int rc2;
                if ((rc2 = idbuf.ensure(sizeof(BoxMeta) * nb + sizeof(int) * nb))) return rc2;
                BoxMeta* d_bm = (BoxMeta*)idbuf.p;
                int* d_kb = (int*)(d_bm + nb);
                HIPCHK(hipMemcpyAsync(d_bm, bm.data(), sizeof(BoxMeta) * nb, hipMemcpyHostToDevice, s));
                const size_t shm = (size_t)(np_max + m_max) * sizeof(double) + (size_t)np_max * sizeof(int);
                std::vector<BoxMeta> cmh;   // compact metadata of row-compressed boxes
                if (nb >= kStepBoxes && shm <= 65536) {
                    // many boxes: one workgroup per box
                    launch_cpqr(nb, d_bm, Ymat, L.d_act, L.d_sr, L.d_perm, d_kb, T64, o->tol, tie, m_max, np_max, s);
                } else {
                    // few (or large) boxes: stepped QR, every launch spread over all boxes' columns.
                    // Tall proxy matrices are first reduced to their triangular factor R (same
                    // column norms, pivots and ID in exact arithmetic), so each pivot step
                    // streams min(m, np) rows instead of m.
                    long sum_y = 0, sum_r = 0;
                    int k_max = 0;
                    for (const BoxMeta& M : bm) {
                        sum_y += (long)M.m * M.np;
                        sum_r += (long)std::min(M.m, M.np) * M.np;
                        k_max = std::max(k_max, std::min(M.m, M.np));
                    }
                    const BoxMeta* qmeta = d_bm;
                    double* QY = Ymat;
                    int q_m_max = m_max;
                    // Compress when the matrices are tall and the rows saved over the pivot
                    // steps outweigh the compression: each step streams the trailing block
                    // (about 16 bytes per entry at about 5 TB/s), while the Householder QR costs
                    // about 0.3 ms per 16 columns with the panel in registers (up to 2560 rows),
                    // 4 ms per 32 columns otherwise.  The number of steps is the largest
                    // predicted rank, or a quarter of the widest box without a prediction.
                    int k_est = k_max / 4;
                    if (!bpred.empty()) k_est = *std::max_element(bpred.begin(), bpred.end());
                    const double t_saved = (double)k_est * (double)(sum_y - sum_r) * 16.0 / 5e12;
                    const double t_compress = m_max <= 2560 ? (k_max + 15) / 16 * 0.3e-3 : (k_max + 31) / 32 * 4e-3;
                    // (matrices taller than the update kernel's LDS allows are always compressed)
                    const bool too_tall = (size_t)m_max * sizeof(double) > 65536;
                    const bool tall = too_tall || (sum_y >= 2 * sum_r &&
                                                   (double)sum_y * sizeof(double) >= 32.0 * (1 << 20) &&
                                                   t_saved > t_compress);
                    if (o->row_compression == CBD_ROWS_ALWAYS || (o->row_compression == CBD_ROWS_AUTO && tall)) {
                        cmh = bm;
                        long o_r = 0;
                        q_m_max = 0;
                        for (BoxMeta& M : cmh) {
                            M.m = std::min(M.m, M.np);
                            M.y = o_r;
                            o_r += (long)M.m * M.np;
                            q_m_max = std::max(q_m_max, M.m);
                        }
                        const size_t nv = (size_t)nb * kHqrVbuf(m_max);
                        if ((rc2 = hqrbuf.ensure(sizeof(BoxMeta) * nb +
                                                 sizeof(double) * ((size_t)nb * kHqrTw + o_act + nv + std::max(o_r, 1L)))))
                            return rc2;
                        BoxMeta* d_cm = (BoxMeta*)hqrbuf.p;
                        double* Tw = (double*)(d_cm + nb);
                        double* halpha = Tw + (size_t)nb * kHqrTw;
                        double* Vb = halpha + o_act;
                        double* Rc = Vb + nv;
                        HIPCHK(hipMemcpyAsync(d_cm, cmh.data(), sizeof(BoxMeta) * nb, hipMemcpyHostToDevice, s));
                        launch_hqr(nb, np_max, m_max, k_max, d_bm, Ymat, Tw, halpha, Vb, d_cm, Rc, s);
                        F->hqr_levels++;
                        qmeta = d_cm;
                        QY = Rc;
                    }
                    if ((size_t)q_m_max * sizeof(double) > 65536)
                        return fail(CBD_EARG, "rs_factor_batched: proxy matrix of " + std::to_string(q_m_max) +
                                                  " rows exceeds the LDS of the QR update kernel");
                    if ((rc2 = qrbuf.ensure(sizeof(double) * (3 * o_act + 2 * nb) + sizeof(int) * (o_act + 2 * nb))))
                        return rc2;
                    QrState st;
                    st.norms = (double*)qrbuf.p;
                    st.alpha = st.norms + o_act;
                    st.beta = st.alpha + o_act;
                    st.nu0 = st.beta + nb;
                    st.pv = (int*)(st.nu0 + nb);
                    st.done = st.pv + o_act;
                    st.k = st.done + nb;
                    launch_qr_init(nb, np_max, qmeta, QY, st, s);
                    int jmax = 0;
                    for (const BoxMeta& M : bm) jmax = std::max(jmax, std::min(M.m, M.np));
                    std::vector<int> done(nb);
                    auto all_done = [&](bool& all) -> int {
                        HIPCHK(hipMemcpyAsync(done.data(), st.done, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
                        HIPCHK(hipStreamSynchronize(s));
                        F->host_syncs++;
                        all = true;
                        for (int v : done) all = all && v;
                        return CBD_OK;
                    };
                    // With predicted ranks, the first steps run without checks: up to the largest
                    // predicted rank plus a margin.  The QR's own stopping rule decides every rank;
                    // a box still running after the budget falls back to checked steps.
                    int j = 0;
                    bool all = false;
                    if (!bpred.empty()) {
                        int kmax_pred = 0;
                        for (int kp : bpred) kmax_pred = std::max(kmax_pred, kp);
                        const int budget = std::min(jmax + 1, (kmax_pred * 11 + 9) / 10 + 2);
                        for (; j < budget; ++j) launch_qr_step(nb, np_max, q_m_max, qmeta, QY, st, j, o->tol, tie, s);
                        F->qr_steps += budget;
                        if ((rc2 = all_done(all))) return rc2;
                        if (!all)
                            for (int v : done) F->mispredicted += !v;
                    }
                    for (; !all && j <= jmax; ++j) {
                        launch_qr_step(nb, np_max, q_m_max, qmeta, QY, st, j, o->tol, tie, s);
                        F->qr_steps++;
                        if (j % 8 == 7 && (rc2 = all_done(all))) return rc2;
                    }
                    launch_qr_finish(nb, np_max, qmeta, QY, st, L.d_act, L.d_sr, L.d_perm, d_kb, T64, s);
                }
                HIPCHK(hipMemcpyAsync(kb.data(), d_kb, sizeof(int) * nb, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                F->host_syncs++;
                return CBD_OK;
            };
            std::vector<int> det;   // boxes with the deterministic ID
            if (o->id_sketch) {
                // randomized ID: the CPQR of Z = Omega Y (ell x np, random signs), ell from
                // the box shape; a saturated sketch falls back to the deterministic ID
                std::vector<BoxMeta> zm;
                std::vector<int> zb, zpred;
                std::vector<unsigned long long> keys(nbc);
                std::vector<BoxMeta> zall(L.meta.begin() + b0, L.meta.begin() + b1);
                std::vector<long> boff(nbc, 0);   // offsets of the boxes' sign words
                long o_z = 0, o_bits = 0, mw_max = 0;
                for (int B = b0; B < b1; ++B) {
                    const BoxMeta& M = L.meta[B];
                    const int ell = sketch_rows(M.m, M.np);
                    keys[B - b0] = ((unsigned long long)L.box_sub[B] << 40) | ((unsigned long long)l << 32) |
                                   (unsigned long long)L.box_idx[B];
                    zall[B - b0].m = ell;
                    zall[B - b0].y = o_z;
                    o_z += (long)ell * M.np;
                    boff[B - b0] = o_bits;
                    const long mw = (long)M.m * ((ell + 31) / 32);
                    o_bits += mw;
                    mw_max = std::max(mw_max, mw);
                    if (ell) {
                        sk_ell[B] = ell;
                        zm.push_back(zall[B - b0]);
                        zb.push_back(B);
                        if (!kpred.empty()) zpred.push_back(std::min(kpred[B], ell));
                    } else {
                        det.push_back(B);
                    }
                }
                if (!zb.empty()) {
                    if ((rc = zbuf.ensure(sizeof(BoxMeta) * nbc + sizeof(unsigned long long) * nbc +
                                          sizeof(long) * nbc + sizeof(double) * std::max(o_z, 1L) +
                                          sizeof(unsigned) * std::max(o_bits, 1L))))
                        return rc;
                    BoxMeta* d_zall = (BoxMeta*)zbuf.p;
                    unsigned long long* d_keys = (unsigned long long*)(d_zall + nbc);
                    long* d_boff = (long*)(d_keys + nbc);
                    double* Z = (double*)(d_boff + nbc);
                    unsigned* d_bits = (unsigned*)(Z + std::max(o_z, 1L));
                    HIPCHK(hipMemcpyAsync(d_zall, zall.data(), sizeof(BoxMeta) * nbc, hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(d_keys, keys.data(), sizeof(unsigned long long) * nbc,
                                          hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(d_boff, boff.data(), sizeof(long) * nbc, hipMemcpyHostToDevice, s));
                    launch_sketch(nbc, np_max_c, mw_max, d_meta_c, d_zall, Y, (const int*)nearbuf.p, Q->d_cidx,
                                  P->N, o->sketch_seed, d_keys, d_boff, d_bits, Z, s);
                    std::vector<int> kz;
                    if ((rc = id_batch(zm, Z, zpred, kz))) return rc;
                    for (size_t e = 0; e < zb.size(); ++e) {
                        if (kz[e] > sk_ell[zb[e]] - kSketchOver) {
                            det.push_back(zb[e]);       // saturated sketch
                            sk_ell[zb[e]] = 0;
                            F->sketch_fallbacks++;
                        } else {
                            kall[zb[e]] = kz[e];
                            F->sketched++;
                        }
                    }
                }
                std::sort(det.begin(), det.end());
            } else {
                for (int B = b0; B < b1; ++B) det.push_back(B);
            }
            if (!det.empty()) {
                std::vector<BoxMeta> dm;
                std::vector<int> dpred, kd;
                for (int B : det) {
                    dm.push_back(L.meta[B]);
                    if (!kpred.empty()) dpred.push_back(kpred[B]);
                }
                if ((rc = id_batch(dm, Y, dpred, kd))) return rc;
                for (size_t e = 0; e < det.size(); ++e) kall[det[e]] = kd[e];
            }
            // ranks and skeleton lists of the chunk to the host now (the ID is complete), so
            // that the next level can be planned while this chunk's elimination runs
            L.k.resize(L.nbox);
            L.sr.resize(o_act);
            for (int B = b0; B < b1; ++B) L.k[B] = kall[B];
            const long a0 = L.meta[b0].act, a1 = b1 < L.nbox ? L.meta[b1].act : o_act;
            HIPCHK(hipMemcpyAsync(d_k_c, L.k.data() + b0, sizeof(int) * nbc, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(L.sr.data() + a0, L.d_sr + a0, sizeof(int) * (a1 - a0), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            F->host_syncs++;
        } else if (ci == 0) {
            // root boxes: no compression, k = 0, identity order
            std::vector<int> zeros(L.nbox, 0), ident(o_act);
            for (int B = 0; B < L.nbox; ++B)
                for (int e = 0; e < L.meta[B].np; ++e) ident[L.meta[B].act + e] = e;
            HIPCHK(hipMemcpyAsync(L.d_k, zeros.data(), sizeof(int) * L.nbox, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(L.d_perm, ident.data(), sizeof(int) * o_act, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(L.d_sr, hact.data(), sizeof(int) * o_act, hipMemcpyHostToDevice, s));
            // the host vectors must stay alive until the copies finish
            HIPCHK(hipStreamSynchronize(s));
            F->host_syncs++;
            L.k.assign(L.nbox, 0);
            L.sr = hact;
        }
        launch_box_matrix<R>(PV, nbc, d_meta_c, L.d_act, Q->d_cidx,
                             o_ch ? (const ChildRef<R>*)chbuf.p : nullptr, App, s);
        // boxes with many DOFs: Cholesky and inverse as multi-workgroup launch sequences
        // (lists hold chunk-local box indices)
        std::vector<int> small, big;
        int np_big = 0;
        for (int B = b0; B < b1; ++B) {
            if (L.meta[B].np >= kBigBox) {
                big.push_back(B - b0);
                np_big = std::max(np_big, L.meta[B].np);
            } else {
                small.push_back(B - b0);
            }
        }
        if (big.empty()) {
            launch_eliminate<R>(nbc, d_meta_c, nullptr, L.d_perm, d_k_c, App, T64, Wk, FF, d_status, bf16, s);
        } else {
            if ((rc = listbuf.ensure(sizeof(int) * nbc))) return rc;
            int* d_small = (int*)listbuf.p;
            int* d_big = d_small + small.size();
            keep.emplace_back(small);
            std::vector<int>& lists = keep.back();
            lists.insert(lists.end(), big.begin(), big.end());
            HIPCHK(hipMemcpyAsync(d_small, lists.data(), sizeof(int) * lists.size(), hipMemcpyHostToDevice, s));
            launch_eliminate<R>((int)small.size(), d_meta_c, d_small, L.d_perm, d_k_c, App, T64, Wk, FF,
                                d_status, bf16, s);
            launch_big_schur<R>((int)big.size(), np_big, d_meta_c, d_big, 1, L.d_perm, d_k_c, App, T64, Wk, FF,
                                bf16, s);
            launch_big_cholesky_inverse<R>((int)big.size(), np_big, d_meta_c, d_big, d_k_c, Wk, FF, d_status, s);
            launch_big_schur<R>((int)big.size(), np_big, d_meta_c, d_big, 2, L.d_perm, d_k_c, App, T64, Wk, FF,
                                bf16, s);
        }
        if (cut.size() > 2) {
            // a breakdown names a chunk-local box: check before the next chunk
            int st_c = 0;
            HIPCHK(hipMemcpyAsync(&st_c, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            F->host_syncs++;
            if (st_c) {
                const int B = b0 + st_c - 1;
                return fail(CBD_ENOTSPD, "rs_factor_batched: Cholesky breakdown at level " + std::to_string(l) +
                                             (root ? " (root)" : "") + ", subdomain " +
                                             std::to_string(L.box_sub[B]) + ", box " + std::to_string(L.box_idx[B]));
            }
        }
        }   // chunks
        HIPCHK(hipGetLastError());
        for (size_t B = 0; B < kpred.size(); ++B) {
            F->pred_abs_err += std::abs(kpred[B] - L.k[B]);
            F->pred_count++;
        }
        for (int B = 0; B < L.nbox; ++B) {
            const double np = L.meta[B].np, k = L.k[B], nr = np - k;
            if (!root) {
                const int ell = B < (int)sk_ell.size() ? sk_ell[B] : 0;
                F->flops += ell ? 2.0 * ell * L.meta[B].m * np + cpqr_flops(ell, np, k) : cpqr_flops(L.meta[B].m, np, k);
            }
            F->flops += elim_flops(k, nr);
        }
    }
    // breakdowns (one slot per level; a split level was checked chunk by chunk)
    std::vector<int> status(Lmax + 1, 0);
    HIPCHK(hipMemcpyAsync(status.data(), statbuf.p, sizeof(int) * (Lmax + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    F->host_syncs++;
    for (int l = 0; l <= Lmax; ++l) {
        if (!status[l]) continue;
        const Level& L = F->levels[l];
        const int B = status[l] - 1;
        return fail(CBD_ENOTSPD, "rs_factor_batched: Cholesky breakdown at level " + std::to_string(l) +
                                     (l == Lmax ? " (root)" : "") + ", subdomain " + std::to_string(L.box_sub[B]) +
                                     ", box " + std::to_string(L.box_idx[B]));
    }
    F->S.assign(D, 0);
    const Level& RL = F->levels.back();
    for (int B = 0; B < RL.nbox; ++B) F->S[RL.box_sub[B]] = RL.meta[B].np;
    return CBD_OK;
}

}  // namespace

extern "C" int rs_factor_batched(cbd_problem p, cbd_partition q, const cbd_rs_opts* o, void* stream,
                                 cbd_factor* out) {
    if (!p || !q || !o || !out) return fail(CBD_EARG, "rs_factor_batched: NULL argument");
    if (q->d != p->d || q->n != p->n)
        return fail(CBD_EARG, "rs_factor_batched: partition is for another grid");
    if (p->grid != CBD_GRID_CELL) return fail(CBD_EARG, "rs_factor_batched: RS needs the cell-centred grid");
    if (!o->exact && (o->n_pxy < 1 || !(o->tol >= 0.0) || !(o->proxy_ratio > 0.75)))
        return fail(CBD_EARG, "rs_factor_batched: need n_pxy >= 1, tol >= 0, proxy_ratio > 0.75");
    if (o->precision != CBD_PREC_FP64 && o->precision != CBD_PREC_FP32 && o->precision != CBD_PREC_BF16GEMM)
        return fail(CBD_EARG, "rs_factor_batched: unknown precision");
    hipStream_t s = (hipStream_t)stream;
    auto* F = new cbd_factor_s;
    F->prob = p;
    F->part = q;
    F->prec = o->precision;
    F->esize = o->precision == CBD_PREC_FP64 ? 8 : 4;
    F->prec = o->precision == CBD_PREC_FP64 ? CBD_PREC_FP64 : CBD_PREC_FP32;   // storage precision
    F->tol = o->tol;
    int rc;
    {
        ScopedTimer tm("factor", s);
        rc = o->precision == CBD_PREC_FP64 ? factor_impl<double>(p, q, o, s, F)
                                           : factor_impl<float>(p, q, o, s, F);
    }
    if (rc) {
        (void)hipStreamSynchronize(s);
        delete F;
        return rc;
    }
    *out = F;
    return CBD_OK;
}

extern "C" int rs_factor_free(cbd_factor f) {
    delete f;
    return CBD_OK;
}

extern "C" int rs_factor_stats(cbd_factor f, int* S, int* n_levels, size_t* bytes, double* flops) {
    if (!f) return fail(CBD_EARG, "rs_factor_stats: NULL factor");
    if (S) std::memcpy(S, f->S.data(), sizeof(int) * f->S.size());
    if (n_levels) *n_levels = f->n_compress;
    if (bytes) *bytes = f->bytes;
    if (flops) *flops = f->flops;
    return CBD_OK;
}

extern "C" int rs_factor_level(cbd_factor f, int level, int* n_boxes, int* ranks, int* np, int* sub) {
    if (!f || level < 0 || level >= (int)f->levels.size()) return fail(CBD_EARG, "rs_factor_level: bad level");
    const Level& L = f->levels[level];
    if (n_boxes) *n_boxes = L.nbox;
    for (int B = 0; B < L.nbox; ++B) {
        if (ranks) ranks[B] = L.k[B];
        if (np) np[B] = L.meta[B].np;
        if (sub) sub[B] = L.box_sub[B];
    }
    return CBD_OK;
}

namespace {
int copy_box(cbd_factor f, const Level& L, int B, int* k, int* nr, int* sk, int* rd, double* T,
             double* E, double* Gi, double* Bss) {
    const BoxMeta& M = L.meta[B];
    const int kk = L.k[B], nn = M.np - kk;
    const long off = f->part->subs[M.sub].offset;
    *k = kk;
    *nr = nn;
    for (int e = 0; e < kk; ++e)
        if (sk) sk[e] = (int)(L.sr[M.act + e] - off);
    for (int e = 0; e < nn; ++e)
        if (rd) rd[e] = (int)(L.sr[M.act + kk + e] - off);
    const long cnt = (long)M.np * M.np;
    std::vector<double> buf(cnt);
    if (f->prec == CBD_PREC_FP64) {
        HIPCHK(hipMemcpy(buf.data(), (const double*)L.d_F + M.f, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> fb(cnt);
        HIPCHK(hipMemcpy(fb.data(), (const float*)L.d_F + M.f, sizeof(float) * cnt, hipMemcpyDeviceToHost));
        for (long e = 0; e < cnt; ++e) buf[e] = fb[e];
    }
    const long nt = (long)kk * nn;
    if (T) std::memcpy(T, buf.data(), sizeof(double) * nt);
    if (E) std::memcpy(E, buf.data() + nt, sizeof(double) * nt);
    if (Gi) std::memcpy(Gi, buf.data() + 2 * nt, sizeof(double) * nn * nn);
    if (Bss) std::memcpy(Bss, buf.data() + 2 * nt + (long)nn * nn, sizeof(double) * kk * kk);
    return CBD_OK;
}
}  // namespace

extern "C" int rs_factor_box(cbd_factor f, int i, int level, int box, int* k, int* nr, int* sk, int* rd,
                             double* T, double* E, double* Ginv, double* Bss) {
    if (!f || !k || !nr || level < 0 || level >= f->n_compress)
        return fail(CBD_EARG, "rs_factor_box: bad argument");
    const Level& L = f->levels[level];
    if (i < 0 || i >= (int)L.sub_start.size() || L.sub_start[i] < 0)
        return fail(CBD_EARG, "rs_factor_box: subdomain has no boxes at this level");
    const int nb = (int)f->part->subs[i].levels[level].size();
    if (box < 0 || box >= nb) return fail(CBD_EARG, "rs_factor_box: bad box");
    return copy_box(f, L, L.sub_start[i] + box, k, nr, sk, rd, T, E, Ginv, Bss);
}

extern "C" int rs_factor_root(cbd_factor f, int i, int* S, int* idx, double* Ginv) {
    if (!f || !S) return fail(CBD_EARG, "rs_factor_root: bad argument");
    const Level& L = f->levels.back();
    if (i < 0 || i >= (int)L.sub_start.size() || L.sub_start[i] < 0)
        return fail(CBD_EARG, "rs_factor_root: bad subdomain");
    int k, nr;
    int rc = copy_box(f, L, L.sub_start[i], &k, &nr, nullptr, idx, nullptr, nullptr, Ginv, nullptr);
    *S = nr;
    return rc;
}

// Large root boxes are applied by GEMMs through global buffers instead of LDS.
static bool root_uses_gemm(const Level& L) { return L.root && L.np_max >= kBigBox; }

// Allocate the apply's buffers for nrhs columns ahead of time (stream capture).
static int apply_prepare(cbd_factor f, int nrhs) {
    int rc = f->v.ensure(f->esize * (size_t)f->part->total * nrhs);
    if (rc) return rc;
    const Level& R = f->levels.back();
    if (root_uses_gemm(R)) {
        const size_t b = f->esize * (size_t)R.nbox * R.np_max * nrhs;
        if ((rc = f->t1.ensure(b)) || (rc = f->t2.ensure(b))) return rc;
    }
    return CBD_OK;
}

template <typename R>
static int apply_impl(cbd_factor f, int nrhs, const double* r, double* z, hipStream_t s) {
    cbd_partition_s* Q = f->part;
    int rc = apply_prepare(f, nrhs);
    if (rc) return rc;
    R* v = (R*)f->v.p;
    for (const Level& L : f->levels)
        if (!root_uses_gemm(L) && (size_t)2 * L.np_max * sizeof(R) > 65536)
            return fail(CBD_EARG, "rs_apply: box of " + std::to_string(L.np_max) + " DOFs exceeds the LDS of the apply kernel");
    launch_gather<R>(r, f->prob->N, nrhs, Q->d_cidx, Q->total, v, s);
    const int nl = (int)f->levels.size();
    for (int l = 0; l < nl; ++l) {
        const Level& L = f->levels[l];
        if (root_uses_gemm(L)) {   // forward and backward root solve at once
            launch_root_apply<R>(L.nbox, L.np_max, 0, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nrhs,
                                 (R*)f->t1.p, (R*)f->t2.p, s);
            continue;
        }
        launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nrhs, L.np_max, true, s);
    }
    for (int l = nl - 1; l >= 0; --l) {
        const Level& L = f->levels[l];
        if (root_uses_gemm(L)) continue;
        launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nrhs, L.np_max, false, s);
    }
    launch_scatter<R>(v, nrhs, Q->d_inv_ptr, Q->d_inv_slot, f->prob->N, z, s);
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int rs_apply(cbd_factor f, int nrhs, const double* r, double* z, void* stream) {
    if (!f || !r || !z || nrhs < 1) return fail(CBD_EARG, "rs_apply: bad argument");
    if (r == z) return fail(CBD_EARG, "rs_apply: r and z alias");
    hipStream_t s = (hipStream_t)stream;
    ScopedTimer tm("apply", s);
    return f->prec == CBD_PREC_FP64 ? apply_impl<double>(f, nrhs, r, z, s) : apply_impl<float>(f, nrhs, r, z, s);
}

// ---------------------------------------------------------------------------
// skeleton-rank predictor
// ---------------------------------------------------------------------------
extern "C" int rank_mlp_params(void) { return kMlpParams; }

extern "C" size_t rank_mlp_workspace_bytes(int n) {
    return sizeof(float) * (size_t)(2 + 4 * kMlpWidth) * (size_t)std::max(n, 0);
}

extern "C" int rank_mlp_forward(const float* params, int n, const float* X, float* y, void* stream) {
    if (!params || n < 0 || (n > 0 && (!X || !y))) return fail(CBD_EARG, "rank_mlp_forward: bad argument");
    launch_mlp_forward(params, n, X, y, nullptr, nullptr, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int rank_mlp_loss_grad(const float* params, int n, const float* X, const float* t, float* grad,
                                  float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!params || !X || !t || !grad || !ws || n < 1) return fail(CBD_EARG, "rank_mlp_loss_grad: bad argument");
    if (ws_bytes < rank_mlp_workspace_bytes(n)) return fail(CBD_EARG, "rank_mlp_loss_grad: workspace too small");
    launch_mlp_loss_grad(params, n, X, t, grad, loss, (float*)ws, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int rank_mlp_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                             void* stream) {
    if (!params || !grad || !m || !v || step < 1) return fail(CBD_EARG, "rank_mlp_adam: bad argument");
    launch_mlp_adam(params, grad, m, v, step, lr, (hipStream_t)stream);
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int rs_factor_features(cbd_factor f, int level, int* n_boxes, float* X, int* k) {
    if (!f || !n_boxes || level < 0 || level >= f->n_compress)
        return fail(CBD_EARG, "rs_factor_features: bad argument");
    const Level& L = f->levels[level];
    *n_boxes = L.nbox;
    for (int B = 0; B < L.nbox; ++B) {
        if (X) box_features(level, L.side[B], L.meta[B].np, L.meta[B].nnear, f->tol, f->prob->d,
                            X + (size_t)B * kMlpFeatures);
        if (k) k[B] = L.k[B];
    }
    return CBD_OK;
}

extern "C" int rs_factor_schedule(cbd_factor f, int* host_syncs, int* qr_steps, int* mispredicted,
                                  double* mean_abs_err, int* row_compressed, int* sketched, int* sketch_fallbacks,
                                  int* chunks) {
    if (!f) return fail(CBD_EARG, "rs_factor_schedule: NULL factor");
    if (host_syncs) *host_syncs = f->host_syncs;
    if (qr_steps) *qr_steps = f->qr_steps;
    if (mispredicted) *mispredicted = f->mispredicted;
    if (mean_abs_err) *mean_abs_err = f->pred_count ? f->pred_abs_err / f->pred_count : 0.0;
    if (row_compressed) *row_compressed = f->hqr_levels;
    if (sketched) *sketched = f->sketched;
    if (sketch_fallbacks) *sketch_fallbacks = f->sketch_fallbacks;
    if (chunks) *chunks = f->chunks;
    return CBD_OK;
}

// ---------------------------------------------------------------------------
// PCG
// ---------------------------------------------------------------------------
namespace {
struct PcgWs {
    double *r, *z, *p, *q, *zold, *partial, *rz, *pq, *rr, *rznew, *alpha, *beta, *fn2;
    int* active;
};
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t carve(PcgWs* w, void* base, long N, int nrhs) {
    size_t vec = align256(sizeof(double) * (size_t)N * nrhs);
    size_t sc = align256(sizeof(double) * nrhs);
    size_t off = 0;
    char* b = (char*)base;
    auto take = [&](size_t n) {
        char* p = b ? b + off : nullptr;
        off += n;
        return p;
    };
    double** vecs[5] = {&w->r, &w->z, &w->p, &w->q, &w->zold};
    for (auto v : vecs) *v = (double*)take(vec);
    w->partial = (double*)take(align256(sizeof(double) * (size_t)nrhs * kDotBlocks));
    double** scal[8] = {&w->rz, &w->pq, &w->rr, &w->rznew, &w->alpha, &w->beta, &w->fn2, nullptr};
    for (int i = 0; i < 7; ++i) *scal[i] = (double*)take(sc);
    w->active = (int*)take(align256(sizeof(int) * nrhs));
    return off;
}
}  // namespace

extern "C" size_t pcg_workspace_bytes(long N, int nrhs) {
    PcgWs w;
    return carve(&w, nullptr, N, nrhs);
}

namespace {
// The two launch sequences of a PCG iteration, around the host read of ||r||:
// A: q = A p, alpha = r.z / p.q, u += alpha p, r -= alpha q, r.r
// B: z = M r, beta, p = z + beta p
struct PcgSeq {
    cbd_problem p;
    cbd_factor fac;
    int nrhs, flexible;
    long N, NV;
    PcgWs w;
    double* u;
    int precond(const double* in, double* outv, hipStream_t s) const {
        if (fac) return rs_apply(fac, nrhs, in, outv, s);
        launch_copy(outv, in, NV, s);
        return CBD_OK;
    }
    int fft = 0;
    int seqA(hipStream_t s) const {
        int rc = fft ? kernel_matvec_fft(p, nrhs, w.p, w.q, s) : kernel_matvec(p, nrhs, w.p, w.q, s);
        if (rc) return rc;
        launch_dot(w.p, w.q, N, nrhs, w.partial, w.pq, s);
        launch_pcg_alpha(w.rz, w.pq, w.active, w.alpha, nrhs, s);
        launch_pcg_update_ur(u, w.r, w.p, w.q, w.alpha, N, nrhs, s);
        launch_dot(w.r, w.r, N, nrhs, w.partial, w.rr, s);
        return CBD_OK;
    }
    int seqB(hipStream_t s) const {
        int rc;
        if (flexible) launch_copy(w.zold, w.z, NV, s);
        if ((rc = precond(w.r, w.z, s))) return rc;
        if (flexible) {
            launch_sub(w.q, w.z, w.zold, NV, s);   // q is free until the next matvec
            launch_dot(w.r, w.q, N, nrhs, w.partial, w.rznew, s);
            launch_pcg_beta(w.rznew, w.rz, w.active, w.beta, nrhs, s);
            launch_dot(w.r, w.z, N, nrhs, w.partial, w.rz, s);
        } else {
            launch_dot(w.r, w.z, N, nrhs, w.partial, w.rznew, s);
            launch_pcg_beta(w.rznew, w.rz, w.active, w.beta, nrhs, s);
        }
        launch_pcg_update_p(w.p, w.z, w.beta, N, nrhs, s);
        return CBD_OK;
    }
};

// Capture one launch sequence into an executable graph.
template <typename Fn>
int capture(hipStream_t s, Fn&& fn, hipGraphExec_t* exec) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    g_capturing = true;
    int rc = fn(s);
    g_capturing = false;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return CBD_OK;
}
}  // namespace

extern "C" int pcg_solve(cbd_problem p, cbd_factor fac, int nrhs, const double* f, double* u, double tol,
                         int maxit, int flags, void* ws, size_t ws_bytes, int* iters, double* relres,
                         void* stream) {
    if (!p || !f || !u || !ws || !iters || !relres || nrhs < 1 || maxit < 0)
        return fail(CBD_EARG, "pcg_solve: bad argument");
    if (flags & ~(CBD_PCG_FLEXIBLE | CBD_PCG_GRAPH | CBD_PCG_FFT)) return fail(CBD_EARG, "pcg_solve: unknown flags");
    if ((flags & CBD_PCG_FFT) && !p->fft_P) return fail(CBD_EARG, "pcg_solve: CBD_PCG_FFT needs cbd_fft_prepare");
    const long N = p->N;
    if (ws_bytes < pcg_workspace_bytes(N, nrhs)) return fail(CBD_EARG, "pcg_solve: workspace too small");
    if (fac && fac->prob != p) return fail(CBD_EARG, "pcg_solve: factor belongs to another problem");
    hipStream_t s = (hipStream_t)stream;
    const bool graph = (flags & CBD_PCG_GRAPH) != 0;
    if (graph && s == nullptr) return fail(CBD_EARG, "pcg_solve: graph mode needs a non-default stream");
    PcgSeq q;
    q.p = p;
    q.fac = fac;
    q.nrhs = nrhs;
    q.flexible = (flags & CBD_PCG_FLEXIBLE) != 0;
    q.fft = (flags & CBD_PCG_FFT) != 0;
    q.N = N;
    q.NV = N * nrhs;
    q.u = u;
    carve(&q.w, ws, N, nrhs);
    PcgWs& w = q.w;
    const long NV = q.NV;
    int rc;
    launch_fill(u, 0.0, NV, s);
    launch_copy(w.r, f, NV, s);
    launch_dot(f, f, N, nrhs, w.partial, w.fn2, s);
    std::vector<double> fn2(nrhs), rr(nrhs);
    std::vector<int> active(nrhs);
    HIPCHK(hipMemcpyAsync(fn2.data(), w.fn2, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int n_active = 0;
    for (int c = 0; c < nrhs; ++c) {
        active[c] = fn2[c] > 0.0;
        n_active += active[c];
        iters[c] = 0;
        relres[c] = active[c] ? 1.0 : 0.0;
    }
    HIPCHK(hipMemcpyAsync(w.active, active.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
    if ((rc = q.precond(w.r, w.z, s))) return rc;
    launch_copy(w.p, w.z, NV, s);
    launch_dot(w.r, w.z, N, nrhs, w.partial, w.rz, s);
    hipGraphExec_t gA = nullptr, gB = nullptr;
    auto cleanup = [&]() {
        if (gA) (void)hipGraphExecDestroy(gA);
        if (gB) (void)hipGraphExecDestroy(gB);
    };
    if (graph && maxit > 0 && n_active > 0) {
        // everything a captured launch needs is allocated beforehand
        if (fac && (rc = apply_prepare(fac, nrhs))) return rc;
        HIPCHK(hipStreamSynchronize(s));
        if ((rc = capture(s, [&](hipStream_t cs) { return q.seqA(cs); }, &gA))) {
            cleanup();
            return rc;
        }
        if ((rc = capture(s, [&](hipStream_t cs) { return q.seqB(cs); }, &gB))) {
            cleanup();
            return rc;
        }
    }
    for (int it = 1; it <= maxit && n_active > 0; ++it) {
        if (graph) {
            hipError_t e = hipGraphLaunch(gA, s);
            if (e != hipSuccess) {
                cleanup();
                return fail(CBD_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
        } else if ((rc = q.seqA(s))) {
            return rc;
        }
        HIPCHK(hipMemcpyAsync(rr.data(), w.rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        n_active = 0;
        for (int c = 0; c < nrhs; ++c) {
            if (!active[c]) continue;
            iters[c] = it;
            relres[c] = std::sqrt(rr[c] / fn2[c]);
            if (relres[c] <= tol) active[c] = 0;
            n_active += active[c];
        }
        if (n_active == 0) break;
        HIPCHK(hipMemcpyAsync(w.active, active.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        if (graph) {
            hipError_t e = hipGraphLaunch(gB, s);
            if (e != hipSuccess) {
                cleanup();
                return fail(CBD_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
        } else if ((rc = q.seqB(s))) {
            return rc;
        }
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    cleanup();
    // active[] on the host stays alive until the last async copy is done (synchronized above)
    return n_active > 0 ? CBD_WNOTCONV : CBD_OK;
}
