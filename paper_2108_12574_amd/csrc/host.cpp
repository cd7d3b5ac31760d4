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
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cbd.h"
#include "internal.h"

using namespace cbd;

thread_local long cbd::g_launches = 0;

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
    // FFT matvec state (cbd_fft_prepare): views of the caller's workspace
    int fft_P = 0, fft_logP = 0, fft_pairs = 0;
    double* fft_ghat = nullptr;
    double2* fft_tw = nullptr;
    double2* fft_buf = nullptr;
    ProblemView view() const {
        return ProblemView{d, n, N, pts, diag, w, rs, grid == CBD_GRID_CELL ? 1.0 / n : 1.0 / (n - 1)};
    }
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

namespace {
int fft_size(int n, int* logP) {
    int P = 2, l = 1;
    while (P < 2 * n - 1) {
        P <<= 1;
        ++l;
    }
    if (logP) *logP = l;
    return P;
}
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

extern "C" size_t cbd_fft_workspace_bytes(int d, int n, int max_pairs) {
    if ((d != 2 && d != 3) || n < 2 || max_pairs < 1) return 0;
    const int P = fft_size(n, nullptr);
    size_t vol = 1;
    for (int t = 0; t < d; ++t) vol *= (size_t)P;
    return al256(sizeof(double) * vol) + al256(sizeof(double2) * (P / 2)) + al256(sizeof(double2) * vol * max_pairs);
}

extern "C" int cbd_fft_prepare(cbd_problem p, int max_pairs, void* ws, size_t ws_bytes, void* stream) {
    if (!p || max_pairs < 1 || !ws) return fail(CBD_EARG, "cbd_fft_prepare: bad argument");
    int logP = 0;
    const int P = fft_size(p->n, &logP);
    if (P > 4096) return fail(CBD_EARG, "cbd_fft_prepare: transform length above 4096 (n > 2048)");
    if (((uintptr_t)ws & 255) != 0) return fail(CBD_EARG, "cbd_fft_prepare: ws must be 256-byte aligned");
    if (ws_bytes < cbd_fft_workspace_bytes(p->d, p->n, max_pairs))
        return fail(CBD_EWORKSPACE, "cbd_fft_prepare: workspace too small (need " +
                                        std::to_string(cbd_fft_workspace_bytes(p->d, p->n, max_pairs)) + " bytes)");
    long vol = 1;
    for (int t = 0; t < p->d; ++t) vol *= P;
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)ws;
    p->fft_P = 0;
    p->fft_ghat = (double*)b;
    b += al256(sizeof(double) * vol);
    p->fft_tw = (double2*)b;
    b += al256(sizeof(double2) * (P / 2));
    p->fft_buf = (double2*)b;
    std::vector<double2> tw(P / 2);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < P / 2; ++k) tw[k] = make_double2(std::cos(2.0 * pi * k / P), -std::sin(2.0 * pi * k / P));
    HIPCHK(hipMemcpyAsync(p->fft_tw, tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice, s));
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

extern "C" int cbd_matvec_set_shape(cbd_problem p, int nrhs, int shape) {
    if (!p || nrhs < 1) return fail(CBD_EARG, "cbd_matvec_set_shape: bad argument");
    const bool wide = shape == 8 + 1 || shape == 8 + 2 || shape == 8 + 4;
    if (shape != 1 && shape != 2 && shape != 4 && !wide)
        return fail(CBD_EARG, "cbd_matvec_set_shape: shape must be 1, 2, 4, 9, 10 or 12");
    if (wide && (p->d != 2 || p->n % matvec_rows_per_block(shape) != 0))
        return fail(CBD_EARG, "cbd_matvec_set_shape: 8-wave shapes need a 2D grid whose side is a multiple of "
                              "their rows per workgroup");
    p->mv_rb[matvec_nb(nrhs) - 1] = shape;
    return CBD_OK;
}

extern "C" int cbd_autotune_matvec(cbd_problem p, int nrhs, double* x, double* y, void* stream, int* choice) {
    if (!p || nrhs < 1 || !x || !y || x == y) return fail(CBD_EARG, "cbd_autotune_matvec: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = matvec_nb(nrhs);
    const int cols = std::min(nrhs, 64);
    launch_fill(x, 1.0, p->N * cols, s);
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int best = matvec_default_rb(nb);
    double best_t = 1e300;
    // row blocks per wave 1, 2, 4 with 4 waves per workgroup; on 2D grids also 2, 4 with 8
    const int cand[5] = {1, 2, 4, 8 + 2, 8 + 4};
    for (int rb : cand) {
        if (rb >= 8 && (p->d != 2 || p->n % matvec_rows_per_block(rb) != 0)) continue;
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
        // candidates come in order of rows per workgroup; within 1% of the best time the
        // later one wins (a taller row band reads x fewer times)
        if (per_row < best_t * 1.01) {
            best_t = per_row;
            best = rb;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
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
    std::vector<int> cidx;      // slot -> global index
    // inverse map in CSR form: the slots holding grid point g are inv_slot[inv_ptr[g] ..
    // inv_ptr[g + 1]), in subdomain order (built on first use; host only)
    std::vector<int> inv_ptr, inv_slot;
    std::once_flag inv_once;
    void build_inverse() {
        std::call_once(inv_once, [this] {
            long N = 1;
            for (int t = 0; t < d; ++t) N *= n;
            std::vector<int> cnt(N + 1, 0);
            for (long e = 0; e < total; ++e) cnt[cidx[e] + 1]++;
            for (long g = 0; g < N; ++g) cnt[g + 1] += cnt[g];
            std::vector<int> slot(total), fill(cnt.begin(), cnt.end() - 1);
            for (long e = 0; e < total; ++e) slot[fill[cidx[e]]++] = (int)e;
            inv_ptr = std::move(cnt);
            inv_slot = std::move(slot);
        });
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

// A factorization's share of the caller's workspace.  Persistent arrays (box lists,
// factor slots, the partition's device index maps, the apply's buffers) are taken
// from the bottom; scratch from the top, as a stack that is cut back at every level
// and every chunk of a level.  All work of a factorization is enqueued on one stream,
// so scratch given back is reused only by work enqueued after the work that used it.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, lo = 0, hi = 0, peak = 0;
    size_t short_by = 0;      // a request that did not fit: the bytes missing
    static size_t al(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }
    void init(void* p, size_t bytes) {
        base = (char*)p;
        cap = bytes & ~(size_t)255;
        lo = 0;
        hi = cap;
        peak = 0;
        short_by = 0;
    }
    void track() { peak = std::max(peak, lo + (cap - hi)); }
    size_t free_bytes() const { return hi - lo; }
    void* low(size_t b) {
        b = al(b);
        if (b > hi - lo) {
            short_by = b - (hi - lo);
            return nullptr;
        }
        void* p = base + lo;
        lo += b;
        track();
        return p;
    }
    void* high(size_t b) {
        b = al(b);
        if (b > hi - lo) {
            short_by = b - (hi - lo);
            return nullptr;
        }
        hi -= b;
        track();
        return base + hi;
    }
};

// Scratch buffer of a level or chunk, carved from the top of the arena; growing it
// takes a new region (the old one is given back with the next cut).
// Scratch of the Gram-matrix ID for a batch of nb boxes with o_g = sum n_p^2 Gram
// entries, in a level of o_act active DOFs: G, its offsets, and the panel state.
size_t gram_bytes(long o_g, int nb, long o_act) {
    return Arena::al(sizeof(double) * (size_t)o_g) + Arena::al(sizeof(long) * nb) +
           Arena::al(sizeof(double) * o_act) + Arena::al(sizeof(double) * nb) + 2 * Arena::al(sizeof(int) * o_act) +
           Arena::al(sizeof(int) * (size_t)nb * kPcholPanel) + Arena::al(sizeof(int) * 3 * (size_t)nb);
}

struct ScratchBuf {
    void* p = nullptr;
    size_t bytes = 0;
    Arena* A = nullptr;
    int ensure(size_t b) {
        if (b <= bytes && p) return CBD_OK;
        void* q = A->high(b);
        if (!q)
            return fail(CBD_EWORKSPACE, "rs_factor_batched: workspace too small (" + std::to_string(A->short_by) +
                                            " more bytes needed for scratch)");
        p = q;
        bytes = b;
        return CBD_OK;
    }
    void reset() {
        p = nullptr;
        bytes = 0;
    }
};

// The host side of an eager factorization, kept for rs_factor_capture: the options and
// rank hints it ran with, and every upload and read in order (payloads at 16-byte
// aligned offsets).
struct FactorTape {
    cbd_rs_opts opts{};
    bool has_hint = false;
    std::vector<int> hint;
    std::vector<char> up, rd;
    std::vector<size_t> up_off, up_len, rd_off, rd_len;
    static void add(std::vector<char>& v, std::vector<size_t>& off, std::vector<size_t>& len, const void* p,
                    size_t b) {
        off.push_back(v.size());
        len.push_back(b);
        v.resize(v.size() + ((b + 15) & ~(size_t)15));
        if (b) std::memcpy(v.data() + off.back(), p, b);
    }
};

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
    int apply_cols = 0;                 // the apply sweep's columns per workgroup (0: default)
    int apply_threads = 0;              // and threads per workgroup (256 or 1024; 0: default)
    // device arrays of the level, in the caller's workspace
    BoxMeta* d_meta = nullptr;
    int *d_act = nullptr, *d_sr = nullptr, *d_perm = nullptr, *d_k = nullptr;
    void* d_F = nullptr;
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
    int sketched_pred = 0;    // boxes whose ID came from the rank-sized first sketch
    int sketch_pred_rejected = 0;   // boxes whose rank-sized sketch was not kept
    int chunks = 0;           // level chunks (more than the number of levels when the workspace is bounded)
    int gram_batches = 0;     // batches whose ID came from the pivoted Cholesky of the Gram matrix
    long launches = 0;        // kernel launches of the factorization
    double pred_abs_err = 0.0;
    int pred_count = 0;
    size_t esize;
    std::vector<Level> levels;   // compressed levels, then the root level
    int n_compress = 0;
    std::vector<int> S;
    size_t bytes = 0;
    double flops = 0.0;
    Arena ws;                    // the caller's workspace (the factor views it)
    int *d_cidx = nullptr, *d_inv_ptr = nullptr, *d_inv_slot = nullptr;   // partition maps
    int apply_rhs = 0;           // columns the apply buffers hold
    void *v = nullptr, *t1 = nullptr, *t2 = nullptr;   // apply: local vectors, large-root buffers
    std::vector<int> stage;      // host source of an upload in flight
    std::vector<int> ranks;      // host source of the ranks_out upload
    int* d_stat = nullptr;       // breakdown slots, one per level
    // graph replay (rs_factor_capture / rs_factor_replay)
    std::unique_ptr<FactorTape> tape;
    hipGraphExec_t graph = nullptr;
    char* gws = nullptr;         // flag word, then the device copies of the tape's payloads
    long graph_launches = 0;     // kernels in the graph
    int stale = 0;               // a replay did not reproduce the recording
    ~cbd_factor_s() {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

namespace {

// Every upload to and read from the device of a factorization goes through here.
// EAGER runs them; RECORD runs them and appends them to the tape; CAPTURE (inside a
// stream capture) runs nothing on the host side of the device: an upload becomes a copy
// from the device copy of the recorded payload (after checking that the host plan
// produced the same bytes), and a read returns the recorded bytes and enqueues a check
// of the device value against them.
struct FactorIo {
    enum Mode { EAGER, RECORD, CAPTURE } mode = EAGER;
    FactorTape* tape = nullptr;
    const char* d_up = nullptr;   // CAPTURE: device copies of tape->up and tape->rd
    const char* d_rd = nullptr;
    int* flag = nullptr;          // CAPTURE: set where a read differs
    size_t ui = 0, ri = 0;        // CAPTURE: next upload / read of the tape
    int* syncs = nullptr;         // counter of stream synchronizations
    int plan_differs() const {
        return fail(CBD_EREPLAN, "rs_factor_capture: the host plan differs from the recorded one");
    }
    int up(void* dst, const void* src, size_t b, hipStream_t s) {
        if (!b) return CBD_OK;
        if (mode == CAPTURE) {
            if (ui >= tape->up_len.size() || tape->up_len[ui] != b ||
                std::memcmp(tape->up.data() + tape->up_off[ui], src, b) != 0)
                return plan_differs();
            if (b % 4 != 0 || (uintptr_t)dst % 4 != 0) return fail(CBD_EARG, "rs_factor_capture: unaligned upload");
            launch_copy_words(dst, d_up + tape->up_off[ui], b, s);
            ++ui;
            return CBD_OK;
        }
        if (mode == RECORD) FactorTape::add(tape->up, tape->up_off, tape->up_len, src, b);
        HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyHostToDevice, s));
        return CBD_OK;
    }
    // device src -> host dst, then the host waits for it (and for all work before it).
    // check = false: a read of breakdown slots, which a replay reports by itself
    int rd(void* dst, const void* src, size_t b, hipStream_t s, bool check = true) {
        if (mode == CAPTURE) {
            if (ri >= tape->rd_len.size() || tape->rd_len[ri] != b) return plan_differs();
            if (b % 4 != 0 || (uintptr_t)src % 4 != 0) return fail(CBD_EARG, "rs_factor_capture: unaligned read");
            if (b) std::memcpy(dst, tape->rd.data() + tape->rd_off[ri], b);
            if (b && check) launch_check_words(src, d_rd + tape->rd_off[ri], b, flag, s);
            ++ri;
            return CBD_OK;
        }
        if (b) HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ++*syncs;
        if (mode == RECORD) FactorTape::add(tape->rd, tape->rd_off, tape->rd_len, dst, b);
        return CBD_OK;
    }
    // the host waits for the uploads so far (their host sources may go)
    int sync(hipStream_t s) {
        if (mode == CAPTURE) return CBD_OK;
        HIPCHK(hipStreamSynchronize(s));
        ++*syncs;
        return CBD_OK;
    }
};

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
// Rows of the first sketch from a predicted rank k_p (0: none): 4 k_p + 32 when below the
// shape-based size; its ID is kept when k <= ell / 4.
constexpr int kSketchPredFactor = 4, kSketchPredExtra = 32;
int predicted_sketch_rows(int m, int np, int kp) {
    const int shape = sketch_rows(m, np);
    const int ell = kSketchPredFactor * std::max(kp, 0) + kSketchPredExtra;
    return shape && ell < shape ? ell : 0;
}

double cpqr_flops(double m, double n, double k) {
    return 4.0 * m * n * k - 2.0 * (m + n) * k * k + 4.0 * k * k * k / 3.0;
}
double elim_flops(double k, double nr) {
    // the method's work: B_sr, B_rr (symmetric), Cholesky, E by a triangular solve, B_ss
    // (symmetric).  The explicit G^{-1} this library stores for the apply is its own
    // choice and is not counted.
    return k * k * nr + 2.0 * k * k * nr + 2.0 * nr * nr * k + nr * nr * nr / 3.0 + k * nr * nr + k * k * nr;
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

// Persistent bytes of the workspace for one level's arrays (as factor_impl takes them).
size_t level_bytes(long nbox, long n_act, long n_f, size_t esize) {
    return Arena::al(sizeof(BoxMeta) * nbox) + 3 * Arena::al(sizeof(int) * n_act) + Arena::al(sizeof(int) * nbox) +
           Arena::al(esize * n_f);
}

// Bytes of the apply's buffers for `cols` right-hand sides.
size_t apply_bytes(long total, long root_boxes, int root_np_max, int cols, size_t esize) {
    size_t b = Arena::al(esize * (size_t)total * cols);
    if (root_np_max >= kBigBox) b += 2 * Arena::al(esize * (size_t)root_boxes * root_np_max * cols);
    return b;
}

template <typename R>
int factor_impl(cbd_problem_s* P, cbd_partition_s* Q, const cbd_rs_opts* o, const int* hint, int* ranks_out,
                hipStream_t s, cbd_factor_s* F, FactorIo& io) {
    int rc = CBD_OK;
    io.syncs = &F->host_syncs;
    Arena& A = F->ws;
    auto short_of = [&](const char* what) {
        return fail(CBD_EWORKSPACE, std::string("rs_factor_batched: workspace too small (") + what + ": " +
                                        std::to_string(A.short_by) + " more bytes needed)");
    };
    // the partition's index maps: slot -> point, and point -> slots for the scatter-add
    Q->build_inverse();
    const long N_ = P->N;
    F->d_cidx = (int*)A.low(sizeof(int) * Q->total);
    F->d_inv_ptr = (int*)A.low(sizeof(int) * (N_ + 1));
    F->d_inv_slot = (int*)A.low(sizeof(int) * Q->total);
    if (!F->d_cidx || !F->d_inv_ptr || !F->d_inv_slot) return short_of("partition maps");
    if ((rc = io.up(F->d_cidx, Q->cidx.data(), sizeof(int) * Q->total, s)) ||
        (rc = io.up(F->d_inv_ptr, Q->inv_ptr.data(), sizeof(int) * (N_ + 1), s)) ||
        (rc = io.up(F->d_inv_slot, Q->inv_slot.data(), sizeof(int) * Q->total, s)))
        return rc;
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
    // level-wide scratch (cut back at every level) and chunk scratch (at every chunk)
    ScratchBuf ybuf, wbuf, t64buf, appbuf, nearbuf, chbuf, mlpbuf;
    ScratchBuf qrbuf, listbuf, hqrbuf, idbuf, zbuf, grambuf;
    for (ScratchBuf* b : {&ybuf, &wbuf, &t64buf, &appbuf, &nearbuf, &chbuf, &mlpbuf, &qrbuf, &listbuf, &hqrbuf,
                          &idbuf, &zbuf, &grambuf})
        b->A = &A;
    double* d_dir = (double*)A.low(sizeof(double) * hdir.size());
    if (!d_dir) return short_of("proxy directions");
    if ((rc = io.up(d_dir, hdir.data(), sizeof(double) * hdir.size(), s))) return rc;

    int Lmax = 0;
    if (!o->exact)
        for (auto& sd : Q->subs) Lmax = std::max(Lmax, sd.root_level);
    F->n_compress = Lmax;
    // one Cholesky-breakdown slot per level, read once at the end: the host plans a
    // level while the previous level's elimination runs
    int* d_stat = (int*)A.low(sizeof(int) * (Lmax + 1));
    if (!d_stat) return short_of("status slots");
    F->d_stat = d_stat;
    F->stage.assign(Lmax + 1, 0);   // kept alive with the factor until the copy is done
    if ((rc = io.up(d_stat, F->stage.data(), sizeof(int) * (Lmax + 1), s))) return rc;
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
    long hint_off = 0;   // first entry of the current level in hint[]

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
        // the previous level's scratch is given back: its work is enqueued before any of
        // this level's
        A.hi = A.cap;
        for (ScratchBuf* b : {&ybuf, &wbuf, &t64buf, &appbuf, &nearbuf, &chbuf, &mlpbuf, &qrbuf, &listbuf, &hqrbuf,
                              &idbuf, &zbuf, &grambuf})
            b->reset();
        // device arrays of the level (kept for the apply), in the order level_bytes counts them
        L.d_meta = (BoxMeta*)A.low(sizeof(BoxMeta) * L.nbox);
        L.d_act = L.d_meta ? (int*)A.low(sizeof(int) * o_act) : nullptr;
        L.d_sr = L.d_act ? (int*)A.low(sizeof(int) * o_act) : nullptr;
        L.d_perm = L.d_sr ? (int*)A.low(sizeof(int) * o_act) : nullptr;
        L.d_k = L.d_perm ? (int*)A.low(sizeof(int) * L.nbox) : nullptr;
        L.d_F = L.d_k ? A.low(sizeof(R) * o_f) : nullptr;
        if (!L.d_F) return short_of(("factor arrays of level " + std::to_string(l)).c_str());
        F->bytes += sizeof(R) * (size_t)o_f;
        // The level's boxes go through the proxy matrices, IDs and elimination in chunks
        // of consecutive boxes whose scratch (Y, elimination work, FP64 T, box matrices)
        // fits what is left of the workspace (and opts->workspace_bytes); the factor
        // arrays stay level-wide.  The level's scratch buffers are sized once, for the
        // largest chunk.
        std::vector<int> cut;
        long my = 1, mf = 1, ma = 1;
        size_t need = 0;
        double hqr = 0.0, zb = 0.0, gb = 0.0;
        {
            auto est = [&](const BoxMeta& M) {
                const double yb = (double)std::max((long)M.m * M.np, (long)M.np * M.np + kScratchCols * M.np);
                const double fb = (double)M.np * M.np;
                return yb * (sizeof(double) + sizeof(R)) + fb * (sizeof(double) + sizeof(R));
            };
            auto al = [](double b) { return Arena::al((size_t)b); };
            const bool sk = o->id_sketch != 0 && !root;
            double budget = std::min((double)A.free_bytes(),
                                     o->workspace_bytes ? (double)o->workspace_bytes : 1e300);
            for (;;) {
                cut.assign(1, 0);
                double acc = 0.0;
                for (int B = 0; B < L.nbox; ++B) {
                    const double e = est(L.meta[B]);
                    if (B > cut.back() && acc + e > budget) {
                        cut.push_back(B);
                        acc = 0.0;
                    }
                    acc += e;
                }
                cut.push_back(L.nbox);
                // exact scratch of this cut: level-wide buffers for the largest chunk
                my = mf = ma = 1;
                hqr = zb = gb = 0.0;
                for (size_t c = 0; c + 1 < cut.size(); ++c) {
                    long cy = 0, cf = 0, o_r = 0, o_z = 0, o_bits = 0;
                    int mmax = 0;
                    const int nb = cut[c + 1] - cut[c];
                    for (int B = cut[c]; B < cut[c + 1]; ++B) {
                        const BoxMeta& M = L.meta[B];
                        cy += std::max((long)M.m * M.np, (long)M.np * M.np + kScratchCols * M.np);
                        cf += (long)M.np * M.np;
                        o_r += (long)std::min(M.m, M.np) * M.np;
                        mmax = std::max(mmax, M.m);
                        const int ell = sk ? sketch_rows(M.m, M.np) : 0;
                        o_z += (long)ell * M.np;
                        o_bits += (long)M.m * ((ell + 31) / 32);
                    }
                    my = std::max(my, cy);
                    mf = std::max(mf, cf);
                    ma = std::max(ma, cf);
                    // row compression runs only in the stepped QR (few boxes, or matrices too
                    // large for one workgroup's LDS)
                    int npmax = 0;
                    for (int B = cut[c]; B < cut[c + 1]; ++B) npmax = std::max(npmax, L.meta[B].np);
                    const size_t shm = (size_t)(npmax + mmax) * sizeof(double) + (size_t)npmax * sizeof(int);
                    if (!root && o->row_compression != CBD_ROWS_NEVER && (nb < kStepBoxes || shm > 65536))
                        hqr = std::max(hqr, (double)sizeof(BoxMeta) * nb +
                                                8.0 * ((double)nb * kHqrTw + o_act + (double)nb * kHqrVbuf(mmax) +
                                                       std::max(o_r, 1L)));
                    if (!root && o->id_method == CBD_ID_GRAM) {
                        long o_g = 0;
                        for (int B = cut[c]; B < cut[c + 1]; ++B) o_g += (long)L.meta[B].np * L.meta[B].np;
                        gb = std::max(gb, (double)gram_bytes(o_g, nb, o_act));
                    }
                    if (sk)
                        zb = std::max(zb, (double)(sizeof(BoxMeta) + 8 + 8) * nb + 8.0 * std::max(o_z, 1L) +
                                              4.0 * std::max(o_bits, 1L));
                }
                need = al(8.0 * my) + al((double)sizeof(R) * my) + al(8.0 * mf) + al((double)sizeof(R) * ma) +
                       al(4.0 * std::max(o_near, 1L)) + al((double)sizeof(ChildRef<R>) * std::max(o_ch, 1L)) +
                       (o->mlp && !root ? al(4.0 * L.nbox * (kMlpFeatures + 1)) : 0) +
                       al(8.0 * (3.0 * o_act + 2.0 * L.nbox) + 4.0 * (o_act + 2.0 * L.nbox)) +
                       al((double)(sizeof(BoxMeta) + 4) * L.nbox) + al(4.0 * L.nbox) + (hqr > 0 ? al(hqr) : 0) + (sk ? al(zb) : 0) +
                       (gb > 0 ? al(gb) : 0);
                if (need <= A.free_bytes()) break;
                if ((int)cut.size() - 1 >= L.nbox) {
                    A.short_by = need - A.free_bytes();
                    return short_of(("scratch of level " + std::to_string(l)).c_str());
                }
                budget *= 0.7;
            }
            if ((rc = ybuf.ensure(sizeof(double) * my)) || (rc = wbuf.ensure(sizeof(R) * my)) ||
                (rc = t64buf.ensure(sizeof(double) * mf)) || (rc = appbuf.ensure(sizeof(R) * ma)) ||
                (rc = nearbuf.ensure(sizeof(int) * std::max(o_near, 1L))) ||
                (rc = chbuf.ensure(sizeof(ChildRef<R>) * std::max(o_ch, 1L))) ||
                (o->mlp && !root && (rc = mlpbuf.ensure(sizeof(float) * (size_t)L.nbox * (kMlpFeatures + 1)))) ||
                (rc = qrbuf.ensure(sizeof(double) * (3 * o_act + 2 * L.nbox) + sizeof(int) * (o_act + 2 * L.nbox))) ||
                (rc = idbuf.ensure((sizeof(BoxMeta) + sizeof(int)) * L.nbox)) ||
                (rc = listbuf.ensure(sizeof(int) * L.nbox)) || (hqr > 0 && (rc = hqrbuf.ensure((size_t)hqr))) || (gb > 0 && (rc = grambuf.ensure((size_t)gb))) ||
                (sk && (rc = zbuf.ensure((size_t)zb))))
                return rc;
        }
        F->chunks += (int)cut.size() - 1;
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
        if ((rc = io.up(L.d_meta, L.meta.data(), sizeof(BoxMeta) * L.nbox, s)) ||
            (rc = io.up(L.d_act, hact.data(), sizeof(int) * o_act, s)) ||
            (rc = io.up(nearbuf.p, hnear.data(), sizeof(int) * o_near, s)) ||
            (rc = io.up(chbuf.p, hch.data(), sizeof(ChildRef<R>) * o_ch, s)))
            return rc;
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
            if ((rc = io.up(dX, feats.data(), sizeof(float) * feats.size(), s))) return rc;
            launch_mlp_forward(o->mlp, L.nbox, dX, dy, nullptr, nullptr, s);
            if ((rc = io.rd(yhat.data(), dy, sizeof(float) * L.nbox, s))) return rc;
            kpred.resize(L.nbox);
            for (int B = 0; B < L.nbox; ++B) {
                const int kmax = std::min(L.meta[B].m, L.meta[B].np);
                const double kp = std::exp2((double)yhat[B]) - 1.0;
                kpred[B] = std::max(0, std::min(kmax, (int)std::lround(std::isfinite(kp) ? kp : (double)kmax)));
            }
        }
        if (!root && hint) {
            // ranks of an earlier factorization of the same layout: the same use as predictions
            kpred.resize(L.nbox);
            for (int B = 0; B < L.nbox; ++B)
                kpred[B] = std::max(0, std::min(std::min(L.meta[B].m, L.meta[B].np), hint[hint_off + B]));
        }
        if (!root) hint_off += L.nbox;
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
        int* d_status = d_stat + l;
        if (!root) {
            launch_proxy_matrix<double>(PV, nbc, d_meta_c, L.d_act, (const int*)nearbuf.p, F->d_cidx,
                                        d_dir, npxy, Y, s);
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
                if ((rc2 = io.up(d_bm, bm.data(), sizeof(BoxMeta) * nb, s))) return rc2;
                const size_t shm = (size_t)(np_max + m_max) * sizeof(double) + (size_t)np_max * sizeof(int);
                std::vector<BoxMeta> cmh;   // compact metadata of row-compressed boxes
                const bool reg = cpqr_reg_fits(m_max, np_max);
                const bool onewg = !reg && nb >= kStepBoxes && shm <= 65536;
                const bool gram = o->id_method == CBD_ID_GRAM && pchol_panel_lds(np_max) <= pchol_panel_lds_limit();
                if (gram) {
                    // the ID from the pivoted Cholesky of G = Y^T Y, by panels of kPcholPanel
                    // pivots (one launch pair per panel)
                    std::vector<long> goffs(nb);
                    long o_g = 0;
                    for (int i = 0; i < nb; ++i) {
                        goffs[i] = o_g;
                        o_g += (long)bm[i].np * bm[i].np;
                    }
                    const size_t gbytes = gram_bytes(o_g, nb, o_act);
                    if ((rc2 = grambuf.ensure(gbytes))) return rc2;
                    char* gp = (char*)grambuf.p;
                    double* Gm = (double*)gp;
                    gp += Arena::al(sizeof(double) * (size_t)o_g);
                    long* d_goff = (long*)gp;
                    gp += Arena::al(sizeof(long) * nb);
                    GramState gs;
                    gs.rdiag = (double*)gp;
                    gp += Arena::al(sizeof(double) * o_act);
                    gs.nu0 = (double*)gp;
                    gp += Arena::al(sizeof(double) * nb);
                    gs.pv = (int*)gp;
                    gp += Arena::al(sizeof(int) * o_act);
                    gs.pos = (int*)gp;
                    gp += Arena::al(sizeof(int) * o_act);
                    gs.piv = (int*)gp;
                    gp += Arena::al(sizeof(int) * (size_t)nb * kPcholPanel);
                    gs.done = (int*)gp;
                    gs.k = gs.done + nb;
                    gs.jend = gs.k + nb;
                    if ((rc2 = io.up(d_goff, goffs.data(), sizeof(long) * nb, s))) return rc2;
                    launch_gram(nb, np_max, d_bm, Ymat, d_goff, Gm, s);
                    int jmax = 0;
                    for (const BoxMeta& M : bm) jmax = std::max(jmax, std::min(M.m, M.np));
                    // panels before the first check: enough for the largest predicted rank
                    // (with a margin), else two
                    int first = 2;
                    if (!bpred.empty()) {
                        const int kp = *std::max_element(bpred.begin(), bpred.end());
                        first = ((kp * 11 + 9) / 10 + 2 + kPcholPanel - 1) / kPcholPanel;
                    }
                    std::vector<int> done(nb);
                    int panels = 0;
                    for (int j0 = 0; j0 <= jmax; j0 += kPcholPanel) {
                        launch_pchol_panel(nb, np_max, d_bm, d_goff, Gm, gs, j0, o->tol, tie, s);
                        ++panels;
                        if (panels < first && j0 + kPcholPanel <= jmax) continue;
                        if ((rc2 = io.rd(done.data(), gs.done, sizeof(int) * nb, s))) return rc2;
                        bool all = true;
                        for (int v : done) all = all && v;
                        if (all) break;
                    }
                    F->qr_steps += panels;
                    F->gram_batches++;
                    launch_pchol_finish(nb, np_max, d_bm, d_goff, Gm, gs, Ymat, L.d_act, L.d_sr, L.d_perm, d_kb, T64,
                                        s);
                } else if (reg) {
                    // small boxes: the whole matrix in one workgroup's registers
                    launch_cpqr_reg(nb, np_max, m_max, d_bm, Ymat, L.d_act, L.d_sr, L.d_perm, d_kb, T64, o->tol, tie,
                                    s);
                } else if (onewg) {
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
                        if ((rc2 = io.up(d_cm, cmh.data(), sizeof(BoxMeta) * nb, s))) return rc2;
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
                        int rc3;
                        if ((rc3 = io.rd(done.data(), st.done, sizeof(int) * nb, s))) return rc3;
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
                return io.rd(kb.data(), d_kb, sizeof(int) * nb, s);
            };
            std::vector<int> det;   // boxes with the deterministic ID
            if (o->id_sketch) {
                // randomized ID: the CPQR of Z = Omega Y (ell x np, random signs).  With a
                // predicted rank k_p, a first sketch of 4 k_p + 32 rows, kept if k <= ell / 4;
                // then the shape-based sketch, kept unless saturated (k > ell - 8); then the
                // deterministic ID
                std::vector<unsigned long long> keys(nbc);
                for (int B = b0; B < b1; ++B)
                    keys[B - b0] = ((unsigned long long)L.box_sub[B] << 40) | ((unsigned long long)l << 32) |
                                   (unsigned long long)L.box_idx[B];
                // one pass over `boxes` (ell_of: sketch rows per chunk box); boxes whose ID is
                // not accepted go to `rejected`
                auto sketch_pass = [&](const std::vector<int>& boxes, const std::vector<int>& ell_of, bool pred,
                                       std::vector<int>& rejected) -> int {
                    std::vector<BoxMeta> zall(L.meta.begin() + b0, L.meta.begin() + b1), zm;
                    std::vector<long> boff(nbc, 0);   // offsets of the boxes' sign words
                    std::vector<int> zpred;
                    for (BoxMeta& Z : zall) Z.m = 0;
                    long o_z = 0, o_bits = 0, mw_max = 0;
                    for (int B : boxes) {
                        const BoxMeta& M = L.meta[B];
                        const int ell = ell_of[B - b0];
                        zall[B - b0].m = ell;
                        zall[B - b0].y = o_z;
                        o_z += (long)ell * M.np;
                        boff[B - b0] = o_bits;
                        const long mw = (long)M.m * ((ell + 31) / 32);
                        o_bits += mw;
                        mw_max = std::max(mw_max, mw);
                        zm.push_back(zall[B - b0]);
                        if (!kpred.empty()) zpred.push_back(std::min(kpred[B], ell));
                    }
                    if (boxes.empty()) return CBD_OK;
                    int rc3;
                    if ((rc3 = zbuf.ensure(sizeof(BoxMeta) * nbc + sizeof(unsigned long long) * nbc +
                                           sizeof(long) * nbc + sizeof(double) * std::max(o_z, 1L) +
                                           sizeof(unsigned) * std::max(o_bits, 1L))))
                        return rc3;
                    BoxMeta* d_zall = (BoxMeta*)zbuf.p;
                    unsigned long long* d_keys = (unsigned long long*)(d_zall + nbc);
                    long* d_boff = (long*)(d_keys + nbc);
                    double* Z = (double*)(d_boff + nbc);
                    unsigned* d_bits = (unsigned*)(Z + std::max(o_z, 1L));
                    if ((rc3 = io.up(d_zall, zall.data(), sizeof(BoxMeta) * nbc, s)) ||
                        (rc3 = io.up(d_keys, keys.data(), sizeof(unsigned long long) * nbc, s)) ||
                        (rc3 = io.up(d_boff, boff.data(), sizeof(long) * nbc, s)))
                        return rc3;
                    launch_sketch(nbc, np_max_c, mw_max, d_meta_c, d_zall, Y, (const int*)nearbuf.p, F->d_cidx,
                                  P->N, o->sketch_seed, d_keys, d_boff, d_bits, Z, s);
                    std::vector<int> kz;
                    if ((rc3 = id_batch(zm, Z, zpred, kz))) return rc3;   // synchronizes: the uploads are done
                    for (size_t e = 0; e < boxes.size(); ++e) {
                        const int B = boxes[e], ell = ell_of[B - b0];
                        const bool ok = pred ? kSketchPredFactor * kz[e] <= ell : kz[e] <= ell - kSketchOver;
                        if (ok) {
                            kall[B] = kz[e];
                            sk_ell[B] = ell;
                            F->sketched++;
                            F->sketched_pred += pred;
                        } else {
                            rejected.push_back(B);
                            F->sketch_pred_rejected += pred;
                        }
                    }
                    return CBD_OK;
                };
                std::vector<int> ell_p(nbc, 0), ell_s(nbc, 0), pass1, pass2;
                for (int B = b0; B < b1; ++B) {
                    const BoxMeta& M = L.meta[B];
                    ell_s[B - b0] = sketch_rows(M.m, M.np);
                    if (!kpred.empty()) ell_p[B - b0] = predicted_sketch_rows(M.m, M.np, kpred[B]);
                    if (ell_p[B - b0]) pass1.push_back(B);
                    else if (ell_s[B - b0]) pass2.push_back(B);
                    else det.push_back(B);
                }
                std::vector<int> rej1, rej2;
                if ((rc = sketch_pass(pass1, ell_p, true, rej1))) return rc;
                pass2.insert(pass2.end(), rej1.begin(), rej1.end());
                std::sort(pass2.begin(), pass2.end());
                if ((rc = sketch_pass(pass2, ell_s, false, rej2))) return rc;
                for (int B : rej2) {
                    det.push_back(B);        // saturated sketch
                    sk_ell[B] = 0;
                    F->sketch_fallbacks++;
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
            if ((rc = io.up(d_k_c, L.k.data() + b0, sizeof(int) * nbc, s)) ||
                (rc = io.rd(L.sr.data() + a0, L.d_sr + a0, sizeof(int) * (a1 - a0), s)))
                return rc;
        } else if (ci == 0) {
            // root boxes: no compression, k = 0, identity order
            std::vector<int> zeros(L.nbox, 0), ident(o_act);
            for (int B = 0; B < L.nbox; ++B)
                for (int e = 0; e < L.meta[B].np; ++e) ident[L.meta[B].act + e] = e;
            if ((rc = io.up(L.d_k, zeros.data(), sizeof(int) * L.nbox, s)) ||
                (rc = io.up(L.d_perm, ident.data(), sizeof(int) * o_act, s)) ||
                (rc = io.up(L.d_sr, hact.data(), sizeof(int) * o_act, s)))
                return rc;
            // the host vectors must stay alive until the copies finish
            if ((rc = io.sync(s))) return rc;
            L.k.assign(L.nbox, 0);
            L.sr = hact;
        }
        launch_box_matrix<R>(PV, nbc, np_max_c, d_meta_c, L.d_act, F->d_cidx,
                             o_ch ? (const ChildRef<R>*)chbuf.p : nullptr, App, s);
        // boxes with many DOFs: Cholesky and inverse as multi-workgroup launch sequences
        // (lists hold chunk-local box indices)
        std::vector<int> small, big;
        int np_big = 0, nr_small = 0;   // largest box of the multi-workgroup path; largest n_r of the others
        for (int B = b0; B < b1; ++B) {
            if (L.meta[B].np >= kBigElim) {
                big.push_back(B - b0);
                np_big = std::max(np_big, L.meta[B].np);
            } else {
                small.push_back(B - b0);
                nr_small = std::max(nr_small, L.meta[B].np - L.k[B]);
            }
        }
        if (big.empty()) {
            launch_eliminate<R>(nbc, d_meta_c, nullptr, L.d_perm, d_k_c, App, T64, Wk, FF, d_status, bf16, nr_small,
                                s);
        } else {
            if ((rc = listbuf.ensure(sizeof(int) * nbc))) return rc;
            int* d_small = (int*)listbuf.p;
            int* d_big = d_small + small.size();
            keep.emplace_back(small);
            std::vector<int>& lists = keep.back();
            lists.insert(lists.end(), big.begin(), big.end());
            if ((rc = io.up(d_small, lists.data(), sizeof(int) * lists.size(), s))) return rc;
            launch_eliminate<R>((int)small.size(), d_meta_c, d_small, L.d_perm, d_k_c, App, T64, Wk, FF,
                                d_status, bf16, nr_small, s);
            launch_big_schur<R>((int)big.size(), np_big, d_meta_c, d_big, 1, L.d_perm, d_k_c, App, T64, Wk, FF,
                                bf16, s);
            launch_big_cholesky_inverse<R>((int)big.size(), np_big, d_meta_c, d_big, d_k_c, Wk, FF, d_status, s);
            launch_big_schur<R>((int)big.size(), np_big, d_meta_c, d_big, 2, L.d_perm, d_k_c, App, T64, Wk, FF,
                                bf16, s);
        }
        if (cut.size() > 2) {
            // a breakdown names a chunk-local box: check before the next chunk (every
            // level so far, so that the lowest failing level is the one reported)
            std::vector<int> st(l + 1, 0);
            if ((rc = io.rd(st.data(), d_stat, sizeof(int) * (l + 1), s, false))) return rc;
            for (int l2 = 0; l2 <= l; ++l2) {
                if (!st[l2]) continue;
                const Level& L2 = F->levels[l2];
                // level l2 < l was not chunked; this level's slot names a box of this chunk
                const int B = (l2 == l ? b0 : 0) + st[l2] - 1;
                return fail(CBD_ENOTSPD, "rs_factor_batched: Cholesky breakdown at level " + std::to_string(l2) +
                                             (L2.root ? " (root)" : "") + ", subdomain " +
                                             std::to_string(L2.box_sub[B]) + ", box " + std::to_string(L2.box_idx[B]));
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
    // the apply's buffers: local vectors of every subdomain for apply_rhs columns, and
    // the box-contiguous buffers of large roots
    A.hi = A.cap;
    {
        const Level& RL = F->levels.back();
        F->apply_rhs = o->apply_rhs > 0 ? o->apply_rhs : 64;
        F->v = A.low(sizeof(R) * (size_t)Q->total * F->apply_rhs);
        if (!F->v) return short_of("apply buffers");
        if (RL.np_max >= kBigBox) {
            const size_t b = sizeof(R) * (size_t)RL.nbox * RL.np_max * F->apply_rhs;
            F->t1 = A.low(b);
            F->t2 = F->t1 ? A.low(b) : nullptr;
            if (!F->t2) return short_of("apply buffers of large roots");
        }
    }
    // ranks of every compressed box, in level and batch order
    if (ranks_out) {
        F->ranks.clear();
        for (int l = 0; l < Lmax; ++l) F->ranks.insert(F->ranks.end(), F->levels[l].k.begin(), F->levels[l].k.end());
        if (!F->ranks.empty())
            HIPCHK(hipMemcpyAsync(ranks_out, F->ranks.data(), sizeof(int) * F->ranks.size(), hipMemcpyHostToDevice, s));
    }
    // breakdowns (one slot per level; a split level was checked chunk by chunk)
    std::vector<int> status(Lmax + 1, 0);
    if ((rc = io.rd(status.data(), d_stat, sizeof(int) * (Lmax + 1), s, false))) return rc;
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

namespace {
int check_factor_args(cbd_problem p, cbd_partition q, const cbd_rs_opts* o, const char* who) {
    if (!p || !q || !o) return fail(CBD_EARG, std::string(who) + ": NULL argument");
    if (q->d != p->d || q->n != p->n) return fail(CBD_EARG, std::string(who) + ": partition is for another grid");
    if (p->grid != CBD_GRID_CELL) return fail(CBD_EARG, std::string(who) + ": RS needs the cell-centred grid");
    if (!o->exact && (o->n_pxy < 1 || !(o->tol >= 0.0) || !(o->proxy_ratio > 0.75)))
        return fail(CBD_EARG, std::string(who) + ": need n_pxy >= 1, tol >= 0, proxy_ratio > 0.75");
    if (o->precision != CBD_PREC_FP64 && o->precision != CBD_PREC_FP32 && o->precision != CBD_PREC_BF16GEMM)
        return fail(CBD_EARG, std::string(who) + ": unknown precision");
    if (o->apply_rhs < 0) return fail(CBD_EARG, std::string(who) + ": negative apply_rhs");
    if (o->id_method != CBD_ID_QR && o->id_method != CBD_ID_GRAM)
        return fail(CBD_EARG, std::string(who) + ": unknown id_method");
    if (o->id_method == CBD_ID_GRAM && !o->exact && !(o->tol >= 1e-7))
        return fail(CBD_EARG, std::string(who) + ": CBD_ID_GRAM needs tol >= 1e-7");
    return CBD_OK;
}

// Boxes of every compressed level in batch order (subdomain by subdomain): at level l,
// subdomain i contributes its partition boxes at l when its root lies above l.
int compressed_levels(const cbd_partition_s* q, const cbd_rs_opts* o) {
    int Lmax = 0;
    if (!o->exact)
        for (auto& sd : q->subs) Lmax = std::max(Lmax, sd.root_level);
    return Lmax;
}
}  // namespace

extern "C" int rs_factor_rank_count(cbd_partition q, const cbd_rs_opts* o, int* count) {
    if (!q || !o || !count) return fail(CBD_EARG, "rs_factor_rank_count: NULL argument");
    const int Lmax = compressed_levels(q, o);
    long c = 0;
    for (int l = 0; l < Lmax; ++l)
        for (auto& sd : q->subs)
            if (sd.root_level > l) c += (long)sd.levels[l].size();
    *count = (int)c;
    return CBD_OK;
}

extern "C" int rs_factor_workspace(cbd_problem p, cbd_partition q, const cbd_rs_opts* o, const int* rank_hint,
                                   size_t* bytes) {
    int rc = check_factor_args(p, q, o, "rs_factor_workspace");
    if (rc) return rc;
    if (!bytes) return fail(CBD_EARG, "rs_factor_workspace: bytes is NULL");
    const size_t es = o->precision == CBD_PREC_FP64 ? 8 : 4;
    const int d = p->d, D = (int)q->subs.size();
    const int Lmax = compressed_levels(q, o);
    const int npxy = o->exact ? 0 : o->n_pxy;
    size_t persistent = Arena::al(sizeof(int) * q->total) * 2 + Arena::al(sizeof(int) * (p->N + 1)) +
                        Arena::al(sizeof(double) * std::max(npxy, 1) * d) + Arena::al(sizeof(int) * (Lmax + 1));
    size_t scratch = 0, fixed = 0;   // chunkable scratch of the largest level; per-level lists
    // active DOFs per box, level by level: leaves hold their points; a parent holds
    // the skeletons of its children (hinted ranks, or a guess without hints)
    std::vector<std::vector<long>> np(D);
    for (int i = 0; i < D; ++i)
        for (auto& lf : q->subs[i].leaves) np[i].push_back(lf.count);
    long h = 0;
    // without hints, a box of n_p DOFs is guessed to keep a_d log10(1/tol) n_p^((d-1)/d)
    // skeletons (ranks grow with the box surface and the digits asked for), a_2 = 0.55,
    // a_3 = 0.4; near-field rows are estimated as 6 n_p (2D) or 12 n_p (3D)
    const double digits = std::max(1.0, -std::log10(std::max(o->tol, 1e-300)));
    auto guess = [&](long np_) -> long {
        if (o->exact) return np_;
        const double a = d == 2 ? 0.55 : 0.4;
        return (long)std::ceil(a * digits * std::pow((double)np_, (d - 1.0) / d));
    };
    const double mrow = d == 2 ? 6.0 : 12.0;
    std::vector<std::vector<long>> kk(D);
    for (int l = 0; l <= Lmax; ++l) {
        const bool root = l == Lmax;
        long nbox = 0, n_act = 0, n_f = 0;
        double sc = 0.0;
        for (int i = 0; i < D; ++i) {
            const Sub& sd = q->subs[i];
            if (!root && sd.root_level <= l) continue;
            if (root) {
                long npr = 0;
                if (o->exact) {
                    npr = (long)sd.index.size();
                } else {
                    for (long v : np[i]) npr += v;   // the root box of this subdomain
                }
                nbox += 1;
                n_act += npr;
                n_f += npr * npr;
                sc += (double)(npr * npr) * (2 * 8 + 2 * es) + (double)kScratchCols * npr * (8 + es);
                continue;
            }
            kk[i].assign(np[i].size(), 0);
            for (size_t b = 0; b < np[i].size(); ++b) {
                const long n_ = np[i][b];
                long k = rank_hint ? rank_hint[h++] : guess(n_);
                k = std::max(0L, std::min(n_, k));
                kk[i][b] = k;
                nbox += 1;
                n_act += n_;
                n_f += n_ * n_;
                const double m = npxy + mrow * n_;
                sc += (m * n_ + n_ * n_ + kScratchCols * n_) * (8 + es) + (double)n_ * n_ * (8 + es) + 8.0 * n_ * n_;
            }
            // parents at level l + 1 (or the root): sums of their children's ranks
            if (l + 1 <= sd.root_level) {
                std::vector<long> next(sd.levels[l + 1].size(), 0);
                for (size_t b = 0; b < sd.levels[l].size(); ++b) next[sd.levels[l][b].parent] += kk[i][b];
                np[i] = next;
            }
        }
        persistent += level_bytes(nbox, n_act, n_f, es);
        scratch = std::max(scratch, (size_t)sc);
        // scratch that is level-wide whatever the chunking: near-field and child lists,
        // pivoted-QR state, batch metadata
        fixed = std::max(fixed, (size_t)(4.0 * mrow * n_act + 64.0 * n_act + 512.0 * nbox) + (16u << 10));
    }
    // apply buffers (the root boxes' sizes are the last level's)
    {
        long rb = 0, rnp = 0;
        for (int i = 0; i < D; ++i) {
            long v = 0;
            if (o->exact) v = (long)q->subs[i].index.size();
            else for (long x : np[i]) v += x;
            rb += 1;
            rnp = std::max(rnp, v);
        }
        persistent += apply_bytes(q->total, rb, (int)rnp, o->apply_rhs > 0 ? o->apply_rhs : 64, es);
    }
    if (o->workspace_bytes) scratch = std::min(scratch, (size_t)o->workspace_bytes);
    *bytes = persistent + scratch + fixed + ((size_t)1 << 20);
    return CBD_OK;
}

extern "C" int rs_factor_batched(cbd_problem p, cbd_partition q, const cbd_rs_opts* o, const int* rank_hint,
                                 void* ws, size_t ws_bytes, int* ranks_out, size_t* ws_used, void* stream,
                                 cbd_factor* out) {
    int rc = check_factor_args(p, q, o, "rs_factor_batched");
    if (rc) return rc;
    if (!out || !ws) return fail(CBD_EARG, "rs_factor_batched: NULL argument");
    if (((uintptr_t)ws & 255) != 0) return fail(CBD_EARG, "rs_factor_batched: ws must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    auto* F = new cbd_factor_s;
    F->prob = p;
    F->part = q;
    F->esize = o->precision == CBD_PREC_FP64 ? 8 : 4;
    F->prec = o->precision == CBD_PREC_FP64 ? CBD_PREC_FP64 : CBD_PREC_FP32;   // storage precision
    F->tol = o->tol;
    F->ws.init(ws, ws_bytes);
    {
        ScopedTimer tm("factor", s);
        const long l0 = g_launches;
        try {
            FactorIo io;
            if (o->record) {
                F->tape.reset(new FactorTape);
                F->tape->opts = *o;
                if (rank_hint) {
                    int nh = 0;
                    (void)rs_factor_rank_count(q, o, &nh);
                    F->tape->has_hint = true;
                    F->tape->hint.assign(rank_hint, rank_hint + nh);
                }
                io.mode = FactorIo::RECORD;
                io.tape = F->tape.get();
            }
            rc = o->precision == CBD_PREC_FP64 ? factor_impl<double>(p, q, o, rank_hint, ranks_out, s, F, io)
                                               : factor_impl<float>(p, q, o, rank_hint, ranks_out, s, F, io);
        } catch (const std::bad_alloc&) {
            rc = fail(CBD_ENOMEM, "rs_factor_batched: host allocation failed");
        }
        F->launches = g_launches - l0;
    }
    if (ws_used) *ws_used = rc == CBD_EWORKSPACE ? F->ws.peak + F->ws.short_by : F->ws.peak;
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

namespace {
size_t al16(size_t b) { return (b + 15) & ~(size_t)15; }
constexpr size_t kGwsFlag = 256;   // the check flag's share of gws
}  // namespace

extern "C" size_t rs_factor_graph_bytes(cbd_factor f) {
    if (!f || !f->tape) return 0;
    return kGwsFlag + al16(f->tape->up.size()) + al16(f->tape->rd.size());
}

extern "C" int rs_factor_capture(cbd_factor f, void* gws, size_t gws_bytes, void* stream) {
    if (!f || !gws) return fail(CBD_EARG, "rs_factor_capture: NULL argument");
    if (!f->tape) return fail(CBD_EARG, "rs_factor_capture: the factor was made without opts.record");
    if (f->stale) return fail(CBD_EREPLAN, "rs_factor_capture: the factor is stale (a replay did not match)");
    if (((uintptr_t)gws & 255) != 0) return fail(CBD_EARG, "rs_factor_capture: gws must be 256-byte aligned");
    if (gws_bytes < rs_factor_graph_bytes(f)) return fail(CBD_EARG, "rs_factor_capture: gws too small");
    FactorTape& T = *f->tape;
    hipStream_t s = (hipStream_t)stream;
    char* g = (char*)gws;
    const size_t up_at = kGwsFlag, rd_at = kGwsFlag + al16(T.up.size());
    if (!T.up.empty()) HIPCHK(hipMemcpyAsync(g + up_at, T.up.data(), T.up.size(), hipMemcpyHostToDevice, s));
    if (!T.rd.empty()) HIPCHK(hipMemcpyAsync(g + rd_at, T.rd.data(), T.rd.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (f->graph) {
        (void)hipGraphExecDestroy(f->graph);
        f->graph = nullptr;
    }
    // a second pass over the host side, on a copy of the factor over the same workspace:
    // the same allocations give the same device addresses
    std::unique_ptr<cbd_factor_s> G(new cbd_factor_s);
    G->prob = f->prob;
    G->part = f->part;
    G->esize = f->esize;
    G->prec = f->prec;
    G->tol = f->tol;
    G->ws.init(f->ws.base, f->ws.cap);
    FactorIo io;
    io.mode = FactorIo::CAPTURE;
    io.tape = &T;
    io.d_up = g + up_at;
    io.d_rd = g + rd_at;
    io.flag = (int*)g;
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{cs};
    hipGraph_t graph = nullptr;
    const long l0 = g_launches;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    g_capturing = true;
    int rc = CBD_OK;
    try {
        launch_set_word(io.flag, 0, cs);
        const int* hint = T.has_hint ? T.hint.data() : nullptr;
        rc = f->prec == CBD_PREC_FP64 ? factor_impl<double>(f->prob, f->part, &T.opts, hint, nullptr, cs, G.get(), io)
                                      : factor_impl<float>(f->prob, f->part, &T.opts, hint, nullptr, cs, G.get(), io);
    } catch (const std::bad_alloc&) {
        rc = fail(CBD_ENOMEM, "rs_factor_capture: host allocation failed");
    }
    g_capturing = false;
    e = hipStreamEndCapture(cs, &graph);
    if (!rc && (io.ui != T.up_len.size() || io.ri != T.rd_len.size())) rc = io.plan_differs();
    // the second pass must have laid the factor out exactly as the first
    if (!rc) {
        bool same = G->ws.lo == f->ws.lo && G->levels.size() == f->levels.size() && G->v == f->v &&
                    G->t1 == f->t1 && G->d_stat == f->d_stat;
        for (size_t l = 0; same && l < f->levels.size(); ++l)
            same = G->levels[l].d_F == f->levels[l].d_F && G->levels[l].d_meta == f->levels[l].d_meta &&
                   G->levels[l].nbox == f->levels[l].nbox;
        if (!same) rc = io.plan_differs();
    }
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&f->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        f->graph = nullptr;
        return fail(CBD_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    f->gws = g;
    f->graph_launches = g_launches - l0;
    return CBD_OK;
}

extern "C" int rs_factor_replay(cbd_factor f, void* stream) {
    if (!f) return fail(CBD_EARG, "rs_factor_replay: NULL factor");
    if (!f->graph) return fail(CBD_EARG, "rs_factor_replay: no graph (rs_factor_capture first)");
    if (f->stale) return fail(CBD_EREPLAN, "rs_factor_replay: the factor is stale (a replay did not match)");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipGraphLaunch(f->graph, s));
    const int nst = (int)f->stage.size();
    std::vector<int> st(nst + 1, 0);
    HIPCHK(hipMemcpyAsync(st.data(), f->gws, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(st.data() + 1, f->d_stat, sizeof(int) * nst, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // reads that differ come first: after one, the plan no longer fits the data and any
    // breakdown may follow from that
    if (st[0]) {
        f->stale = 1;
        return fail(CBD_EREPLAN, "rs_factor_replay: the factorization read values other than the recorded ones "
                                 "(ranks, skeletons or stop flags changed); factor again");
    }
    for (int l = 0; l < nst; ++l) {
        if (!st[l + 1]) continue;
        f->stale = 1;
        const Level& L = f->levels[l];
        const int B = st[l + 1] - 1;
        return fail(CBD_ENOTSPD, "rs_factor_replay: Cholesky breakdown at level " + std::to_string(l) +
                                     (L.root ? " (root)" : "") + ", subdomain " +
                                     std::to_string(B < L.nbox ? L.box_sub[B] : -1) + ", box " +
                                     std::to_string(B < L.nbox ? L.box_idx[B] : -1));
    }
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

// z = sum_i R_i^T A_i^{-1} R_i r over the subdomains whose slots lie in [s0, s1) (all of
// them: the whole range), in blocks of at most apply_rhs columns.
template <typename R>
static int apply_impl(cbd_factor f, int nrhs, const double* r, double* z, long s0, long s1, hipStream_t s) {
    R* v = (R*)f->v;
    for (const Level& L : f->levels)
        if (!root_uses_gemm(L) && (size_t)2 * L.np_max * sizeof(R) > apply_level_lds_limit<R>())
            return fail(CBD_EARG, "rs_apply: box of " + std::to_string(L.np_max) + " DOFs exceeds the LDS of the apply kernel");
    const long N = f->prob->N;
    const int nl = (int)f->levels.size();
    for (int c0 = 0; c0 < nrhs; c0 += f->apply_rhs) {
        const int nc = std::min(f->apply_rhs, nrhs - c0);
        const double* rc = r + (long)c0 * N;
        double* zc = z + (long)c0 * N;
        launch_gather<R>(rc, N, nc, f->d_inv_ptr, f->d_inv_slot, s0, s1, v, s);
        for (int l = 0; l < nl; ++l) {
            const Level& L = f->levels[l];
            if (root_uses_gemm(L)) {   // forward and backward root solve at once
                launch_root_apply<R>(L.nbox, L.np_max, 0, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nc,
                                     (R*)f->t1, (R*)f->t2, s);
                continue;
            }
            launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nc, L.np_max, L.apply_cols,
                                  L.apply_threads, true, s);
        }
        for (int l = nl - 1; l >= 0; --l) {
            const Level& L = f->levels[l];
            if (root_uses_gemm(L)) continue;
            launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nc, L.np_max, L.apply_cols,
                                  L.apply_threads, false, s);
        }
        launch_scatter<R>(v, nc, f->d_inv_ptr, f->d_inv_slot, N, zc, s);
    }
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

// cbd_autotune_apply: each level's candidates timed by forward and backward sweeps of
// that level on the factor's local vectors (filled by a gather of r).
template <typename R>
static int autotune_apply_impl(cbd_factor f, int nrhs, const double* r, hipStream_t s, int* choices) {
    cbd_partition_s* Q = f->part;
    R* v = (R*)f->v;
    const long N = f->prob->N;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    const size_t lim = apply_level_lds_limit<R>();
    for (size_t l = 0; l < f->levels.size(); ++l) {
        Level& L = f->levels[l];
        if (choices) choices[2 * l] = choices[2 * l + 1] = 0;
        if (root_uses_gemm(L) || L.nbox == 0) continue;
        int best = 0, best_nt = 0;
        float best_t = 0.f;
        for (int cand = 0; cand < 12; ++cand) {
            const int cols = 8 << (cand & 3), nt = 256 << (cand >> 2);
            if (cols > nrhs && cols != 8) continue;
            if ((size_t)2 * L.np_max * cols * sizeof(R) > lim) continue;
            auto sweep = [&]() {
                launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nrhs, L.np_max, cols, nt,
                                      true, s);
                launch_apply_level<R>(L.nbox, L.d_meta, L.d_sr, L.d_k, (const R*)L.d_F, v, nrhs, L.np_max, cols, nt,
                                      false, s);
            };
            // one warm-up and three timed sweeps, each from freshly gathered vectors (repeated
            // sweeps would scale them up by the inverse's norm every time)
            float ms = 0.f;
            for (int rep = 0; rep < 4; ++rep) {
                launch_gather<R>(r, N, nrhs, f->d_inv_ptr, f->d_inv_slot, 0, Q->total, v, s);
                HIPCHK(hipEventRecord(e0, s));
                sweep();
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                if (rep) ms += t;
            }
            // within 2% of the best counts as a tie, which goes to the earlier candidate
            // (fewer columns and threads per workgroup)
            if (!best || ms < best_t * 0.98f) {
                best = cols;
                best_nt = nt;
                best_t = ms;
            }
        }
        L.apply_cols = best;
        L.apply_threads = best_nt;
        if (choices) {
            choices[2 * l] = best;
            choices[2 * l + 1] = best_nt;
        }
    }
    HIPCHK(hipGetLastError());
    return CBD_OK;
}

extern "C" int cbd_autotune_apply(cbd_factor f, int nrhs, const double* r, void* stream, int* choices) {
    if (!f || !r || nrhs < 1) return fail(CBD_EARG, "cbd_autotune_apply: bad argument");
    if (nrhs > f->apply_rhs) return fail(CBD_EARG, "cbd_autotune_apply: nrhs exceeds the factor's apply_rhs");
    if (f->stale) return fail(CBD_EREPLAN, "cbd_autotune_apply: the factor is stale (a replay did not match)");
    hipStream_t s = (hipStream_t)stream;
    return f->prec == CBD_PREC_FP64 ? autotune_apply_impl<double>(f, nrhs, r, s, choices)
                                    : autotune_apply_impl<float>(f, nrhs, r, s, choices);
}

extern "C" int cbd_apply_set_shape(cbd_factor f, int level, int cols, int threads) {
    if (!f || level < 0 || level >= (int)f->levels.size()) return fail(CBD_EARG, "cbd_apply_set_shape: bad level");
    if (cols != 0 && cols != 8 && cols != 16 && cols != 32 && cols != 64)
        return fail(CBD_EARG, "cbd_apply_set_shape: cols must be 0, 8, 16, 32 or 64");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(CBD_EARG, "cbd_apply_set_shape: threads must be 0, 256, 512 or 1024");
    Level& L = f->levels[level];
    const size_t es = f->prec == CBD_PREC_FP64 ? sizeof(double) : sizeof(float);
    const size_t lim = f->prec == CBD_PREC_FP64 ? apply_level_lds_limit<double>() : apply_level_lds_limit<float>();
    if (cols && (size_t)2 * L.np_max * cols * es > lim)
        return fail(CBD_EARG, "cbd_apply_set_shape: the level's boxes need more LDS at this width");
    L.apply_cols = cols;
    L.apply_threads = threads;
    return CBD_OK;
}

extern "C" int rs_apply(cbd_factor f, int nrhs, const double* r, double* z, void* stream) {
    if (!f || !r || !z || nrhs < 1) return fail(CBD_EARG, "rs_apply: bad argument");
    if (r == z) return fail(CBD_EARG, "rs_apply: r and z alias");
    if (f->stale) return fail(CBD_EREPLAN, "rs_apply: the factor is stale (a replay did not match)");
    hipStream_t s = (hipStream_t)stream;
    ScopedTimer tm("apply", s);
    const long tot = f->part->total;
    return f->prec == CBD_PREC_FP64 ? apply_impl<double>(f, nrhs, r, z, 0, tot, s)
                                    : apply_impl<float>(f, nrhs, r, z, 0, tot, s);
}

extern "C" int rs_apply_sub(cbd_factor f, int i, int nrhs, const double* r, double* z, void* stream) {
    if (!f || !r || !z || nrhs < 1) return fail(CBD_EARG, "rs_apply_sub: bad argument");
    if (r == z) return fail(CBD_EARG, "rs_apply_sub: r and z alias");
    if (f->stale) return fail(CBD_EREPLAN, "rs_apply_sub: the factor is stale (a replay did not match)");
    if (i < 0 || i >= (int)f->part->subs.size()) return fail(CBD_EARG, "rs_apply_sub: bad subdomain");
    hipStream_t s = (hipStream_t)stream;
    const Sub& sd = f->part->subs[i];
    const long s0 = sd.offset, s1 = sd.offset + (long)sd.index.size();
    return f->prec == CBD_PREC_FP64 ? apply_impl<double>(f, nrhs, r, z, s0, s1, s)
                                    : apply_impl<float>(f, nrhs, r, z, s0, s1, s);
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

extern "C" int rank_mlp_loss_grad_noalloc(const float* params, int n, const float* X, const float* t, float* grad,
                                          float* loss, void* stream) {
    if (!params || !X || !t || !grad || n < 1) return fail(CBD_EARG, "rank_mlp_loss_grad_noalloc: bad argument");
    if (n > kMlpStaticMax)
        return fail(CBD_EARG, "rank_mlp_loss_grad_noalloc: " + std::to_string(n) + " samples exceed the limit of " +
                                  std::to_string(kMlpStaticMax));
    float* scr = mlp_static_scratch();
    if (!scr) return fail(CBD_EHIP, "rank_mlp_loss_grad_noalloc: no device address for the library scratch");
    launch_mlp_loss_grad(params, n, X, t, grad, loss, scr, (hipStream_t)stream);
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
                                  int* chunks, int* sketched_pred, int* sketch_pred_rejected, long* launches) {
    if (!f) return fail(CBD_EARG, "rs_factor_schedule: NULL factor");
    if (launches) *launches = f->launches;
    if (host_syncs) *host_syncs = f->host_syncs;
    if (qr_steps) *qr_steps = f->qr_steps;
    if (mispredicted) *mispredicted = f->mispredicted;
    if (mean_abs_err) *mean_abs_err = f->pred_count ? f->pred_abs_err / f->pred_count : 0.0;
    if (row_compressed) *row_compressed = f->hqr_levels;
    if (sketched) *sketched = f->sketched;
    if (sketch_fallbacks) *sketch_fallbacks = f->sketch_fallbacks;
    if (chunks) *chunks = f->chunks;
    if (sketched_pred) *sketched_pred = f->sketched_pred;
    if (sketch_pred_rejected) *sketch_pred_rejected = f->sketch_pred_rejected;
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
    if (fac && fac->stale) return fail(CBD_EREPLAN, "pcg_solve: the factor is stale (a replay did not match)");
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
    // the executable graphs are destroyed on every return path
    struct Graphs {
        hipGraphExec_t a = nullptr, b = nullptr;
        ~Graphs() {
            if (a) (void)hipGraphExecDestroy(a);
            if (b) (void)hipGraphExecDestroy(b);
        }
    } graphs;
    hipGraphExec_t& gA = graphs.a;
    hipGraphExec_t& gB = graphs.b;
    if (graph && maxit > 0 && n_active > 0) {
        HIPCHK(hipStreamSynchronize(s));
        if ((rc = capture(s, [&](hipStream_t cs) { return q.seqA(cs); }, &gA))) return rc;
        if ((rc = capture(s, [&](hipStream_t cs) { return q.seqB(cs); }, &gB))) return rc;
    }
    for (int it = 1; it <= maxit && n_active > 0; ++it) {
        if (graph) {
            hipError_t e = hipGraphLaunch(gA, s);
            if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
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
            if (e != hipSuccess) return fail(CBD_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        } else if ((rc = q.seqB(s))) {
            return rc;
        }
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(s));
    // active[] on the host stays alive until the last async copy is done (synchronized above)
    return n_active > 0 ? CBD_WNOTCONV : CBD_OK;
}
