// Host runtime behind the C ABI of include/rpa.h: validation, G-sphere and
// index tables, pair lists, workspace management and the launch sequence of
// Table 1 steps 3-13 (orbitals, pair densities, PAW, optical row, weights,
// grouped rank-k update, Cholesky log-determinant, frequency sum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <optional>
#include <string>
#include <vector>

#include "../../include/rpa.h"
#include "internal.hpp"

using namespace rpa;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(RPA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr double kDeltaF = 1e-8;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Device scratch of the allocation-free entry point (rpa_ec_noalloc): every workspace of that call is
// carved out of this array, one copy per device, held until the process ends. Host code never uses its
// name as an address: rpa_create looks up each device's copy once with hipGetSymbolAddress and keeps the
// pointer in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device; filled under g_scratch_mu

// the device's scratch address (device must be current); looked up once per device
int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RPA_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return RPA_OK;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct rpa_ctx {
    int device = 0;
    double A[3][3];
    double B[3][3];
    int N[3];
    double volume = 0;
    size_t cap = 0;
    size_t used = 0;
    FftPlan plan[3];
    std::map<std::string, DevBuf> bufs;
    // pinned staging for per-call host tables, released by an event
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t staged = nullptr;
    bool staged_valid = false;
    // failure flags of the last E_c evaluation (device int[nw])
    int* last_fail = nullptr;
    int last_nw = 0;
    // stage profiler: start/end events recorded on the launch stream
    bool prof = false;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    double prof_ms[16] = {0};
    long long prof_n[16] = {0};
    int last_nq = 0;
    std::vector<int> last_qorder;   // caller's q index of each job of the last E_c evaluation
    // rank-k update variant per (precision, padded NG): 1 = 64x64 tiles, 4 / 5 = pipelined 64x128 tiles
    // with FP64 accumulation
    // (4: four waves, 5: eight waves per workgroup)
    std::map<uint64_t, int> tune;
    std::map<uint64_t, double> tune_ms;
    // the captured batch graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint64_t graph_key = 0;
    bool capturing = false;
    bool pair_reg = true;   // register-resident pair transforms where supported
    int max_chunk = 0;      // upper bound on the pairs of one chunk (0: set by the workspace budget alone)
    int paw_win = 0;        // upper bound on the bands m of one MFMA PAW pass (0: set by the Z buffer's size)
    bool autotune = true;   // split precisions: time the rank-k variants for each new sphere-size bucket
    // arena mode (rpa_ec_noalloc): workspaces are carved from the device scratch instead of hipMalloc'd, and
    // host tables are staged in ordinary host memory instead of a pinned arena
    void* scratch = nullptr;            // this device's scratch (set at rpa_create)
    char* arena = nullptr;              // non-null while a call runs in arena mode
    size_t arena_cap = 0, arena_off = 0;
    std::map<std::string, DevBuf> abufs;
    std::vector<char> host_stage;
    // non-blocking stream the batch sequence is captured on (the legacy default stream cannot be)
    hipStream_t cap_stream = nullptr;
    // look-ahead of the blocked Cholesky: the trailing update of each step runs on
    // la_stream and the rows below the next diagonal block on la2_stream, beside the
    // main stream's panel and solve (default priority, non-blocking)
    hipStream_t la_stream = nullptr;
    hipStream_t la2_stream = nullptr;
    hipEvent_t la_ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t la2_ev[3] = {nullptr, nullptr, nullptr};
};

namespace {

// ---------------------------------------------------------------- profiler
enum Stage {
    S_ORB = 0, S_PAIR_XY, S_PAIR_Z, S_PAW, S_OPTICAL, S_WEIGHTS, S_PACK, S_HERK, S_CHOL,
    S_BW_INV, S_BW_GEMM, S_BW_PAIRS, S_BW_REST, S_COUNT
};
const char* kStageNames[S_COUNT] = {"orbitals", "pair_xy", "pair_z_gather", "paw", "optical", "weights",
                                    "split_pack", "herk", "cholesky", "adjoint_inverse", "adjoint_gemm",
                                    "adjoint_pairs", "adjoint_rest"};

hipEvent_t prof_event(rpa_ctx* c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    rpa_ctx* c;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(rpa_ctx* c_, int st, hipStream_t s_) : c(c_), stage(st), s(s_) {
        if (c->prof && !c->capturing && (a = prof_event(c))) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = prof_event(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->recs.push_back({stage, a, b});
    }
};

void prof_collect(rpa_ctx* c) {
    for (auto& r : c->recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_ms[r.stage] += ms;
            c->prof_n[r.stage] += 1;
        }
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
}

// ---------------------------------------------------------------- tuning / graphs
uint64_t tune_key(rpa_precision p, int NGp) { return ((uint64_t)(uint32_t)p << 32) | (uint32_t)NGp; }

void drop_graph(rpa_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_key = 0;
}

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
    template <typename V> void val(const V& v) { bytes(&v, sizeof(v)); }
};

// ---------------------------------------------------------------- buffers
int get_buf(rpa_ctx* c, const char* name, size_t bytes, hipStream_t s, void** out) {
    if (c->arena) {
        DevBuf& a = c->abufs[name];
        if (a.p && a.bytes >= bytes) {
            *out = a.p;
            return RPA_OK;
        }
        const size_t want = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
        if (c->arena_off + want > c->arena_cap)
            return fail(RPA_ERR_NOMEM, std::string("workspace ") + name + " does not fit the device scratch of " +
                                           std::to_string(c->arena_cap) + " bytes (" +
                                           std::to_string(c->arena_off + want) + " needed so far)");
        a.p = c->arena + c->arena_off;
        a.bytes = want;
        c->arena_off += want;
        *out = a.p;
        return RPA_OK;
    }
    DevBuf& b = c->bufs[name];
    if (b.bytes >= bytes && b.p) {
        *out = b.p;
        return RPA_OK;
    }
    if (b.p) {
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipFree(b.p));
        c->used -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    const size_t want = std::max<size_t>(bytes, 256);
    if (c->cap && c->used + want > c->cap)
        return fail(RPA_ERR_NOMEM, std::string("workspace cap exceeded by buffer ") + name);
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(RPA_ERR_NOMEM, std::string("hipMalloc failed for ") + name);
    }
    b.bytes = want;
    c->used += want;
    *out = b.p;
    return RPA_OK;
}

// One pinned arena per call: host tables are packed into it and copied with a
// single hipMemcpyAsync on the caller's stream; the next call waits for that
// copy before reusing the arena.
struct Upload {
    struct Item {
        const void* src;
        size_t bytes;
        size_t off;
        void** dst;
    };
    std::vector<Item> items;
    size_t total = 0;
    template <typename V>
    void add(const std::vector<V>& v, void** dst) {
        items.push_back({v.data(), v.size() * sizeof(V), total, dst});
        total += (v.size() * sizeof(V) + 255) & ~size_t(255);
    }
};

int do_upload(rpa_ctx* c, Upload& u, hipStream_t s, const char* bufname) {
    if (u.total == 0) return RPA_OK;
    if (c->staged_valid) HIP_TRY(hipEventSynchronize(c->staged));
    if (c->arena) {
        // arena mode: ordinary host memory, kept until the copy's event has completed
        if (c->host_stage.size() < u.total) c->host_stage.resize(u.total);
        void* dev = nullptr;
        int rc = get_buf(c, bufname, u.total, s, &dev);
        if (rc) return rc;
        for (auto& it : u.items) {
            if (it.bytes) std::memcpy(c->host_stage.data() + it.off, it.src, it.bytes);
            *it.dst = static_cast<char*>(dev) + it.off;
        }
        HIP_TRY(hipMemcpyAsync(dev, c->host_stage.data(), u.total, hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(c->staged, s));
        c->staged_valid = true;
        return RPA_OK;
    }
    if (c->pinned_bytes < u.total) {
        if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_bytes = 0;
        HIP_TRY(hipHostMalloc(&c->pinned, u.total, hipHostMallocDefault));
        c->pinned_bytes = u.total;
    }
    void* dev = nullptr;
    int rc = get_buf(c, bufname, u.total, s, &dev);
    if (rc) return rc;
    for (auto& it : u.items) {
        if (it.bytes) std::memcpy(static_cast<char*>(c->pinned) + it.off, it.src, it.bytes);
        *it.dst = static_cast<char*>(dev) + it.off;
    }
    HIP_TRY(hipMemcpyAsync(dev, c->pinned, u.total, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(c->staged, s));
    c->staged_valid = true;
    return RPA_OK;
}

// ------------------------------------------------------------- geometry
void reciprocal(const double A[3][3], double B[3][3]) {
    // B = 2 pi inv(A)^T via cofactors
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double inv[3][3];
    inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = kTwoPi * inv[j][i];
}

double det3(const double A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

// |shift + m.B|^2 summed in a fixed order (no contraction: see build flags)
double kvec(const double B[3][3], const double* shift, const int32_t* m, double* k) {
    for (int c = 0; c < 3; ++c) k[c] = ((shift[c] + m[0] * B[0][c]) + m[1] * B[1][c]) + m[2] * B[2][c];
    return (k[0] * k[0] + k[1] * k[1]) + k[2] * k[2];
}

int check_grid(const rpa_cell* cell, FftPlan* plans) {
    for (int i = 0; i < 3; ++i) {
        if (cell->n[i] < 2 || !make_plan(cell->n[i], &plans[i]))
            return fail(RPA_ERR_UNSUPPORTED, "grid length " + std::to_string(cell->n[i]) +
                                                 " is not a product of 2, 3 and 5 (and >= 2)");
    }
    if ((long long)cell->n[0] * cell->n[1] > 65535LL)
        return fail(RPA_ERR_UNSUPPORTED, "N1*N2 above 65535 is not supported");
    if (!(std::fabs(det3(cell->A)) > 0)) return fail(RPA_ERR_INPUT, "singular cell");
    return RPA_OK;
}

// ------------------------------------------------------------ validation
int nproj_total(const rpa_states* s) { return s->natoms > 0 ? s->proj_off[s->natoms] : 0; }

int check_states(const rpa_ctx* c, const rpa_states* s, const char* tag) {
    const std::string t(tag);
    if (!s) return fail(RPA_ERR_INPUT, t + ": NULL state set");
    if (s->nbands <= 0 || s->nQ <= 0) return fail(RPA_ERR_SHAPE, t + ": nbands and nQ must be positive");
    if (!s->miller || !s->C || !s->eps || !s->f) return fail(RPA_ERR_INPUT, t + ": NULL miller, C, eps or f");
    if (s->natoms < 0) return fail(RPA_ERR_SHAPE, t + ": negative natoms");
    if (s->natoms > 0) {
        if (!s->proj_off) return fail(RPA_ERR_INPUT, t + ": NULL proj_off");
        if (s->proj_off[0] != 0) return fail(RPA_ERR_SHAPE, t + ": proj_off[0] must be 0");
        for (int a = 0; a < s->natoms; ++a)
            if (s->proj_off[a + 1] <= s->proj_off[a]) return fail(RPA_ERR_SHAPE, t + ": proj_off not increasing");
        if (!s->P) return fail(RPA_ERR_INPUT, t + ": NULL P");
    }
    for (int i = 0; i < s->nQ; ++i)
        for (int d = 0; d < 3; ++d) {
            const int m = s->miller[3 * i + d];
            if (2 * std::abs(m) >= c->N[d])
                return fail(RPA_ERR_ALIAS, t + ": plane-wave Miller index outside the grid");
        }
    for (int n = 0; n < s->nbands; ++n) {
        if (!(s->f[n] >= 0.0 && s->f[n] <= 2.0)) return fail(RPA_ERR_INPUT, t + ": occupation outside [0, 2]");
        if (s->dfde && !(s->dfde[n] >= 0.0 && std::isfinite(s->dfde[n])))
            return fail(RPA_ERR_INPUT, t + ": -df/de negative or not finite");
        if (!std::isfinite(s->eps[n])) return fail(RPA_ERR_INPUT, t + ": non-finite eigenvalue");
        if (n > 0 && s->eps[n] < s->eps[n - 1]) return fail(RPA_ERR_INPUT, t + ": eigenvalues not ascending");
        if (n > 0 && s->f[n] > s->f[n - 1] + kDeltaF)
            return fail(RPA_ERR_INPUT, t + ": occupations increase with energy");
    }
    return RPA_OK;
}

int max_abs_miller(const int32_t* m, int n, int d) {
    int r = 0;
    for (int i = 0; i < n; ++i) r = std::max(r, std::abs(m[3 * i + d]));
    return r;
}

bool same_set(const rpa_states* a, const rpa_states* b) {
    return a == b || (a->C == b->C && a->P == b->P && a->nbands == b->nbands && a->nQ == b->nQ &&
                      a->miller == b->miller);
}

// ------------------------------------------------------------- per-q plan
struct QPlan {
    PairGeom g;
    int NG = 0, NGp = 0, g0 = -1;
    std::vector<int32_t> kx, ky, col_start, col_g, col_kz;
    // the same entries over the columns that hold any (the forward z pass transforms only those)
    std::vector<int32_t> zcol, zcol_start, zcol_kz;
    std::vector<double> vsqrt;
};

// Miller ranges of a sphere along each axis
void sphere_box(const rpa_qspec* qs, int lo[3], int hi[3]) {
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = qs->gmiller[d];
    for (int i = 0; i < qs->NG; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], (int)qs->gmiller[3 * i + d]);
            hi[d] = std::max(hi[d], (int)qs->gmiller[3 * i + d]);
        }
}

// box (optional): {lo1, hi1, lo2, hi2}, the (m1, m2) columns the pair transform keeps when several q-points
// share it; the sphere's own extent otherwise
int plan_q(rpa_ctx* c, const rpa_qspec* qs, QPlan& P, bool need_coulomb, const int* box = nullptr) {
    if (!qs) return fail(RPA_ERR_INPUT, "NULL qspec");
    if (qs->NG <= 0 || !qs->gmiller) return fail(RPA_ERR_SHAPE, "empty G-sphere");
    const int NG = qs->NG;
    int lo[3], hi[3];
    sphere_box(qs, lo, hi);
    if (box) {
        lo[0] = box[0];
        hi[0] = box[1];
        lo[1] = box[2];
        hi[1] = box[3];
    }
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] + 1 > c->N[d]) return fail(RPA_ERR_ALIAS, "G-sphere wider than the grid");
    PairGeom& g = P.g;
    g.N1 = c->N[0];
    g.N2 = c->N[1];
    g.N3 = c->N[2];
    g.K1 = hi[0] - lo[0] + 1;
    g.K2 = hi[1] - lo[1] + 1;
    g.ncols = g.K1 * g.K2;
    g.NG = NG;
    g.NGp = (NG + kTile - 1) / kTile * kTile;
    g.p1 = c->plan[0];
    g.p2 = c->plan[1];
    g.p3 = c->plan[2];
    P.NG = NG;
    P.NGp = g.NGp;
    P.kx.resize(g.K1);
    P.ky.resize(g.K2);
    for (int i = 0; i < g.K1; ++i) P.kx[i] = ((lo[0] + i) % g.N1 + g.N1) % g.N1;
    for (int i = 0; i < g.K2; ++i) P.ky[i] = ((lo[1] + i) % g.N2 + g.N2) % g.N2;
    g.x0 = P.kx[0];
    g.y0 = P.ky[0];
    g.K3 = hi[2] - lo[2] + 1;
    g.z0 = ((lo[2] % g.N3) + g.N3) % g.N3;
    // entries sorted by column (m1, m2); value = G index, (kz << 16) | column
    std::vector<int> order(NG);
    std::vector<int> col(NG);
    for (int i = 0; i < NG; ++i) {
        const int32_t* m = qs->gmiller + 3 * i;
        col[i] = (m[1] - lo[1]) * g.K1 + (m[0] - lo[0]);
    }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return col[a] < col[b]; });
    P.col_start.assign(g.ncols + 1, 0);
    for (int i = 0; i < NG; ++i) P.col_start[col[i] + 1]++;
    for (int k = 0; k < g.ncols; ++k) P.col_start[k + 1] += P.col_start[k];
    P.col_g.resize(NG);
    P.col_kz.resize(NG);
    for (int r = 0; r < NG; ++r) {
        const int i = order[r];
        const int kz = ((qs->gmiller[3 * i + 2] % g.N3) + g.N3) % g.N3;
        P.col_g[r] = i;
        P.col_kz[r] = (kz << 16) | col[i];
    }
    std::vector<int32_t> cidx(g.ncols, -1);
    P.zcol.clear();
    P.zcol_start.assign(1, 0);
    for (int k = 0; k < g.ncols; ++k)
        if (P.col_start[k + 1] > P.col_start[k]) {
            cidx[k] = (int32_t)P.zcol.size();
            P.zcol.push_back(k);
            P.zcol_start.push_back(P.col_start[k + 1]);
        }
    g.nzc = (int)P.zcol.size();
    P.zcol_kz.resize(NG);
    for (int r = 0; r < NG; ++r) P.zcol_kz[r] = (P.col_kz[r] & ~0xffff) | cidx[P.col_kz[r] & 0xffff];
    // Coulomb v^1/2 and the G = 0 index
    P.vsqrt.assign(g.NGp, 0.0);
    const double s4pi = std::sqrt(4.0 * kPi);
    for (int i = 0; i < NG; ++i) {
        double k[3];
        const double k2 = kvec(c->B, qs->q, qs->gmiller + 3 * i, k);
        const int32_t* m = qs->gmiller + 3 * i;
        const bool g0 = m[0] == 0 && m[1] == 0 && m[2] == 0;
        if (g0) P.g0 = i;
        if (k2 > 0.0) {
            P.vsqrt[i] = s4pi / std::sqrt(k2);
        } else {
            if (!qs->optical && need_coulomb) return fail(RPA_ERR_INPUT, "q + G = 0 outside the optical limit");
            P.vsqrt[i] = s4pi;
        }
    }
    if (qs->optical) {
        if (qs->q[0] != 0.0 || qs->q[1] != 0.0 || qs->q[2] != 0.0)
            return fail(RPA_ERR_INPUT, "optical limit requires q = 0");
    }
    return RPA_OK;
}

int check_pair(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, const rpa_qspec* qs) {
    int rc = check_states(c, k, "k");
    if (rc) return rc;
    rc = check_states(c, kq, "kq");
    if (rc) return rc;
    if (k->natoms != kq->natoms) return fail(RPA_ERR_SHAPE, "k and kq have different atom counts");
    for (int a = 0; a <= k->natoms && k->natoms > 0; ++a)
        if (k->proj_off[a] != kq->proj_off[a]) return fail(RPA_ERR_SHAPE, "k and kq projector offsets differ");
    if (k->natoms > 0 && !qs->Qpaw) return fail(RPA_ERR_INPUT, "NULL Qpaw with PAW atoms present");
    if (qs->optical && k->natoms > 0 && !qs->Dpaw) return fail(RPA_ERR_INPUT, "optical limit needs Dpaw");
    for (int d = 0; d < 3; ++d) {
        int mg = 0;
        for (int i = 0; i < qs->NG; ++i) mg = std::max(mg, std::abs((int)qs->gmiller[3 * i + d]));
        const int tot = max_abs_miller(k->miller, k->nQ, d) + max_abs_miller(kq->miller, kq->nQ, d) + mg;
        if (tot > c->N[d] - 1)
            return fail(RPA_ERR_ALIAS, "grid axis " + std::to_string(d) + " of " + std::to_string(c->N[d]) +
                                           " points aliases the pair product (|m_k|+|m_kq|+|m_G| = " +
                                           std::to_string(tot) + ")");
    }
    if (qs->optical) {
        if (k->nQ != kq->nQ || std::memcmp(k->miller, kq->miller, sizeof(int32_t) * 3 * k->nQ) != 0)
            return fail(RPA_ERR_SHAPE, "optical limit needs identical plane-wave sets at k and k+q");
    }
    return RPA_OK;
}

int check_freq(const rpa_freq* fr) {
    if (!fr || fr->nw <= 0 || !fr->omega || !fr->weight) return fail(RPA_ERR_INPUT, "empty frequency grid");
    for (int i = 0; i < fr->nw; ++i)
        if (!(fr->omega[i] >= 0.0) || !std::isfinite(fr->weight[i])) return fail(RPA_ERR_INPUT, "bad frequency node");
    return RPA_OK;
}

// transitions n -> m with f_n - f_m > 0 (n outer, or m outer when m_major)
void pair_list(const rpa_states* k, const rpa_states* kq, std::vector<int32_t>& pn, std::vector<int32_t>& pm,
               bool m_major) {
    pn.clear();
    pm.clear();
    const int no = m_major ? kq->nbands : k->nbands, ni = m_major ? k->nbands : kq->nbands;
    for (int o = 0; o < no; ++o)
        for (int i = 0; i < ni; ++i) {
            const int n = m_major ? i : o, m = m_major ? o : i;
            if (k->f[n] - kq->f[m] > kDeltaF) {
                pn.push_back(n);
                pm.push_back(m);
            }
        }
}

// the distinct (x, y) columns of a scatter map, as offsets y * N1 + x into a z-plane, ascending
std::vector<int32_t> grid_columns(const rpa_ctx* c, const std::vector<int32_t>& map) {
    const int32_t plane = c->N[0] * c->N[1];
    std::vector<char> used(plane, 0);
    for (int32_t m : map) used[m % plane] = 1;
    std::vector<int32_t> cols;
    for (int32_t i = 0; i < plane; ++i)
        if (used[i]) cols.push_back(i);
    return cols;
}

std::vector<int32_t> scatter_map(const rpa_ctx* c, const rpa_states* s) {
    std::vector<int32_t> map(s->nQ);
    for (int i = 0; i < s->nQ; ++i) {
        int x = ((s->miller[3 * i] % c->N[0]) + c->N[0]) % c->N[0];
        int y = ((s->miller[3 * i + 1] % c->N[1]) + c->N[1]) % c->N[1];
        int z = ((s->miller[3 * i + 2] % c->N[2]) + c->N[2]) % c->N[2];
        map[i] = (z * c->N[1] + y) * c->N[0] + x;
    }
    return map;
}

template <typename T>
std::vector<cplx<T>> twiddles(int N) {
    // exp(-2 pi i t/N); in FP32 followed by the low parts fl(value - hi) (twiddle_len entries)
    std::vector<cplx<T>> t(twiddle_len<T>(N));
    for (int i = 0; i < N; ++i) {
        const double a = kTwoPi * i / N;
        const double c = std::cos(a), sn = -std::sin(a);
        t[i] = mk(T(c), T(sn));
        if (sizeof(T) == 4) t[N + i] = mk(T(c - (double)t[i].x), T(sn - (double)t[i].y));
    }
    return t;
}

// ------------------------------------------------------------ the engine
// One call = one Batch: tables shared by every q (frequencies, twiddles, PAW
// offsets), one KSet per (k, k+q) state-set pair (pair list, index maps,
// eigenvalues) and one QJob per q-point (sphere tables, Coulomb, chi0
// accumulator, rank-k kernel variant). Planning and uploads happen first; the
// kernel sequence afterwards touches only pre-sized buffers, so it can be
// captured into a graph.
struct KSet {
    const rpa_states* k;
    const rpa_states* kq;
    std::vector<int32_t> pn, pm;
    std::vector<int32_t> mapk, mapkq;
    std::vector<int32_t> zcolk, zcolkq;   // (x, y) columns of the grid that hold coefficients, y * N1 + x
    std::vector<double> epsk, epskq, fk, fkq;
    std::vector<int32_t> nlist_all;  // n = 0 .. nbands-1
    std::vector<int32_t> drude_band; // bands with -df/de > 0 (intraband head at q -> 0) and their -df/de
    std::vector<double> drude_mdf;
    void* d_drude_band = nullptr; void* d_drude_mdf = nullptr;
    void* d_pn = nullptr; void* d_pm = nullptr;
    void* d_mapk = nullptr; void* d_mapkq = nullptr;
    void* d_zcolk = nullptr; void* d_zcolkq = nullptr;
    void* d_epsk = nullptr; void* d_epskq = nullptr; void* d_fk = nullptr; void* d_fkq = nullptr;
    void* d_nlist = nullptr;
};

// The pairs of every chunk of one k set grouped by band n (stable), for the n-factorised MFMA PAW term:
// perm[p0 + i] is the chunk-local index of its i-th pair in that order, seg holds per segment of at most 64
// pairs of one band (n - n_lo, first, count), and chunk c's segments are seg[3 s0_c ..], n_lo_c its lowest n.
struct PawN {
    std::vector<int32_t> perm, seg;
    std::vector<int32_t> s0, ns, nlo, nn;   // per chunk
    void* d_perm = nullptr;
    void* d_seg = nullptr;
};

struct QJob {
    const rpa_qspec* qs = nullptr;
    QPlan qp;
    void* d_kx = nullptr; void* d_ky = nullptr; void* d_cs = nullptr; void* d_cg = nullptr; void* d_ckz = nullptr;
    void* d_zc = nullptr; void* d_zcs = nullptr; void* d_zckz = nullptr;
    void* d_vs = nullptr;
    // optical limit: plane-wave momentum weights per k set and qhat.D
    std::vector<std::vector<double>> wq;
    std::vector<void*> d_wq;
    std::vector<double> Dq;
    void* d_Dq = nullptr;
    int variant = 0;   // 0 FP64 MFMA, 1 split 64x64, 4 / 5 split 64x128 pipelined (four / eight waves)
    int Pc = 0;        // pair chunk
    double* cr = nullptr;
    double* ci = nullptr;
    double* ec = nullptr;
    double* F = nullptr;
    bool fresh = false;   // the accumulator holds nothing yet (no update has run into it)
    int ld = 0;           // leading dimension of this q-point's chi0 / -K matrices (its class's)
    int orig = 0;         // index of this q-point in the caller's list (jobs are ordered by class)
    int k0 = 0, k1 = -1;  // the (k, k+q) sets of this q-point: B.ks[k0 .. k1-1] (k1 < 0: every set)
    bool uses(size_t ik) const { return k1 < 0 || ((int)ik >= k0 && (int)ik < k1); }
};

// q-points whose matrices share one leading dimension: adjacent jobs q0 .. q0 + nq - 1, accumulators at cr
// (all real parts) and ci (all imaginary parts), one matrix every ld^2 doubles
struct QClass {
    int ld = 0, q0 = 0, nq = 0;
    double* cr = nullptr;
    double* ci = nullptr;
};

// A state set given at k1 of the irreducible zone with a point operation (Eq. kmap, Eq. trans_wfs, Table 1
// steps 4 and 7) becomes a plain state set: its plane-wave labels are transformed on the host, and these
// device jobs, first in the call's launch sequence, conjugate its coefficients (time reversal) and rotate
// its projections.
struct UnfoldJob {
    const double* C_in = nullptr;
    double* C_out = nullptr;      // time reversal only
    size_t nC = 0;
    const double* P_in = nullptr;
    double* P_out = nullptr;
    int nb = 0, nproj = 0, tr = 0;
    std::vector<int32_t> tab;     // per output column: source column base, Np, row offset of its D row
    std::vector<double> D, ph;    // the D blocks; per output column the Bloch phase (re, im)
    void* d_tab = nullptr; void* d_D = nullptr; void* d_ph = nullptr;
};

struct Batch {
    rpa_ctx* c = nullptr;
    hipStream_t s = nullptr;
    rpa_precision prec = RPA_FP64;
    int nw = 0;
    std::vector<double> om, ow;
    std::vector<int32_t> qoff, poff;
    std::vector<cplx<double>> tw64[3];
    std::vector<cplx<float>> tw32[3];
    void* d_om = nullptr; void* d_ow = nullptr; void* d_tw[3] = {nullptr, nullptr, nullptr};
    void* d_qoff = nullptr; void* d_poff = nullptr;
    void* d_wq = nullptr;            // q weights (batched calls)
    std::string prefix;              // buffer-name prefix (graph-owned and tuning buffers)
    std::vector<KSet> ks;
    std::vector<QJob> qj;
    bool m_major = false;            // forward chi0: pairs ordered by m, then n (orbital reuse in cache)
    bool allow_paw_mfma = true;      // the adjoint keeps the factorised VALU PAW term (its own tables)
    bool realfreq = false;           // real frequencies w + i eta: nw = 2 nw_user weight rows (Re, Im)
    double eta = 0.0;
    int nw_user = 0;
    bool paw_mfma = false;           // set by presize: PAW correction as an MFMA GEMM per band m
    int paw_mwin = 0;                // set by presize: bands m per MFMA PAW pass (bounds the Z buffer)
    bool paw_nform = false;          // set by presize: the MFMA PAW term factorised per band n (Y_n), not per m
    std::map<std::pair<int, int>, PawN> pawn;  // (k set, chunk size): pair indices of every chunk grouped by n
    bool share_xy = false;           // several q-points with shared sets: one pair transform per chunk for all
    bool allow_share_xy = true;      // the adjoint keeps one q-point's own box
    int ld = 0;                      // the largest leading dimension of the batch's chi0 / -K matrices
    std::vector<QClass> cls;         // the q-points grouped by leading dimension
    std::deque<rpa_states> usets;              // state sets unfolded from the irreducible zone
    std::deque<std::vector<int32_t>> umiller;  // their plane-wave labels
    std::deque<UnfoldJob> ujobs;
    bool fp64() const { return prec == RPA_FP64; }
    size_t elem() const { return fp64() ? sizeof(double) : sizeof(float); }
};

int autotune_run(rpa_ctx* c, rpa_precision prec, int NG, int npairs, int nw, hipStream_t s);

// sphere sizes that share one autotuning result: the padded sphere rounded up to 128 (up to 2048) or 256
int tune_bucket(int NGp) {
    const int g = NGp <= 2048 ? 128 : 256;
    return (NGp + g - 1) / g * g;
}

int default_variant(const rpa_ctx* c, rpa_precision prec, int NGp) {
    if (prec == RPA_FP64) return 0;
    auto it = c->tune.find(tune_key(prec, NGp));
    if (it != c->tune.end()) return it->second;
    return ((NGp + 127) / 128 >= 4) ? 5 : 1;
}

// Leading dimension of a q-point's matrices in a batch of nq: its padded sphere alone, or, with several
// q-points, the padded sphere rounded up to 128 (up to 2048) or 256 (beyond), so that spheres of similar
// size share one batched factorisation at most 1/8 of padding per dimension
int class_ld(int NGp, int nq) {
    if (nq <= 1 || NGp <= 1024) return NGp;
    const int g = NGp <= 2048 ? 128 : 256;
    return (NGp + g - 1) / g * g;
}

int chunk_size(const rpa_ctx* c, const QPlan& qp, int nw, size_t elem, int variant) {
    const PairGeom& g = qp.g;
    const size_t per = (size_t)g.N3 * g.ncols * 2 * elem + 2 * (size_t)g.NGp * elem + (size_t)nw * 8 +
                       (size_t)(g.NGp + 127) / 128 * 128 * 16;
    size_t budget = (size_t)6 << 30;
    if (c->cap) budget = std::min(budget, c->cap / 4);
    if (c->arena) budget = std::min(budget, c->arena_cap / 4);
    size_t pc = budget / per;
    pc = std::max<size_t>(pc, 64);
    pc = std::min<size_t>(pc, 1 << 20);
    if (c->max_chunk > 0) pc = std::min<size_t>(pc, (size_t)c->max_chunk);
    (void)variant;
    return (int)pc;
}

int begin(Batch& B, rpa_ctx* c, const rpa_freq* fr, rpa_precision prec, void* stream) {
    B.c = c;
    B.s = static_cast<hipStream_t>(stream);
    B.prec = prec;
    if (prec != RPA_FP64 && prec != RPA_SPLIT_BF16 && prec != RPA_SPLIT_FP16)
        return fail(RPA_ERR_INPUT, "unknown precision");
    HIP_TRY(hipSetDevice(c->device));
    if (fr) {
        int rc = check_freq(fr);
        if (rc) return rc;
        B.nw = fr->nw;
        B.om.assign(fr->omega, fr->omega + fr->nw);
        B.ow.assign(fr->weight, fr->weight + fr->nw);
    }
    return RPA_OK;
}

// The set at k = (-1)^s T k1 + G0 from the set `s` at k1 and its operation (validated here): labels
// m -> (-1)^s U^-T m - g0 (the coefficient of e^{i G.r} in u_k(r) = e^{-i G0.r} [conj] u_k1(T^-1 r)),
// coefficients conjugated with time reversal, projections P^a_k,i = e^{i k1.L_a} sum_j D^a_ij P^b_k1,j
// (conjugated with time reversal).
int unfold_set(Batch& B, const rpa_states* s, const std::string& tag, Upload& up, const rpa_states** out) {
    rpa_ctx* c = B.c;
    const rpa_symop* o = s->sym;
    const std::string t = tag + ": symmetry operation";
    const int32_t(*U)[3] = o->rot;
    const long long det = (long long)U[0][0] * ((long long)U[1][1] * U[2][2] - (long long)U[1][2] * U[2][1]) -
                          (long long)U[0][1] * ((long long)U[1][0] * U[2][2] - (long long)U[1][2] * U[2][0]) +
                          (long long)U[0][2] * ((long long)U[1][0] * U[2][1] - (long long)U[1][1] * U[2][0]);
    if (det != 1 && det != -1) return fail(RPA_ERR_INPUT, t + ": det U must be +1 or -1");
    if (o->time_reversal != 0 && o->time_reversal != 1) return fail(RPA_ERR_INPUT, t + ": time_reversal not 0 or 1");
    // U^-1 = adj(U) / det
    long long Ui[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            Ui[i][j] = ((long long)U[r0][c0] * U[r1][c1] - (long long)U[r0][c1] * U[r1][c0]) * det;
        }
    // Cartesian T = A^T U A^-T, with A^-1[e][j] = B[j][e] / 2 pi
    double T[3][3];
    for (int a = 0; a < 3; ++a)
        for (int e = 0; e < 3; ++e) {
            double v = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) v += c->A[i][a] * U[i][j] * c->B[j][e] / kTwoPi;
            T[a][e] = v;
        }
    for (int a = 0; a < 3; ++a)
        for (int e = 0; e < 3; ++e) {
            double v = 0.0;
            for (int i = 0; i < 3; ++i) v += T[a][i] * T[e][i];
            if (std::fabs(v - (a == e ? 1.0 : 0.0)) > 1e-9)
                return fail(RPA_ERR_INPUT, t + ": U is not a rotation of this lattice (A^T U A^-T not orthogonal)");
        }
    const double sgn = o->time_reversal ? -1.0 : 1.0;
    double kn = 0.0, kd = 0.0;
    for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        for (int e = 0; e < 3; ++e) v += sgn * T[a][e] * o->kibz[e];
        for (int i = 0; i < 3; ++i) v += o->gshift[i] * c->B[i][a];
        kd = std::max(kd, std::fabs(v - s->kpt[a]));
        kn = std::max(kn, std::fabs(s->kpt[a]));
    }
    if (kd > 1e-9 * (1.0 + kn)) return fail(RPA_ERR_INPUT, t + ": kpt differs from (-1)^s T kibz + G0");
    B.umiller.emplace_back(3 * (size_t)s->nQ);
    std::vector<int32_t>& m2 = B.umiller.back();
    const long long is = o->time_reversal ? -1 : 1;
    for (int q = 0; q < s->nQ; ++q) {
        const int32_t* m = s->miller + 3 * q;
        for (int e = 0; e < 3; ++e)
            m2[3 * q + e] = (int32_t)(is * (Ui[0][e] * m[0] + Ui[1][e] * m[1] + Ui[2][e] * m[2]) - o->gshift[e]);
    }
    rpa_states d = *s;
    d.miller = m2.data();
    d.sym = nullptr;
    B.ujobs.emplace_back();
    UnfoldJob& J = B.ujobs.back();
    J.nb = s->nbands;
    J.tr = o->time_reversal;
    if (o->time_reversal) {
        void* p = nullptr;
        int rc = get_buf(c, (B.prefix + "sym:C:" + tag).c_str(), 16 * (size_t)s->nbands * s->nQ, B.s, &p);
        if (rc) return rc;
        J.C_in = static_cast<const double*>(s->C);
        J.C_out = static_cast<double*>(p);
        J.nC = (size_t)s->nbands * s->nQ;
        d.C = p;
    }
    if (s->natoms > 0) {
        if (!o->atom_map || !o->atom_shift || !o->proj_rot)
            return fail(RPA_ERR_INPUT, t + ": NULL atom_map, atom_shift or proj_rot with PAW atoms present");
        const int na = s->natoms, np_tot = nproj_total(s);
        size_t doff = 0;
        for (int a = 0; a < na; ++a) {
            const int b = o->atom_map[a];
            const int np = s->proj_off[a + 1] - s->proj_off[a];
            if (b < 0 || b >= na) return fail(RPA_ERR_INPUT, t + ": atom_map entry out of range");
            if (s->proj_off[b + 1] - s->proj_off[b] != np)
                return fail(RPA_ERR_SHAPE, t + ": atom_map pairs atoms with different projector counts");
            double L[3];
            for (int e = 0; e < 3; ++e)
                L[e] = o->atom_shift[3 * a] * c->A[0][e] + o->atom_shift[3 * a + 1] * c->A[1][e] +
                       o->atom_shift[3 * a + 2] * c->A[2][e];
            const double arg = o->kibz[0] * L[0] + o->kibz[1] * L[1] + o->kibz[2] * L[2];
            for (int i = 0; i < np; ++i) {
                J.tab.push_back(s->proj_off[b]);
                J.tab.push_back(np);
                J.tab.push_back((int32_t)(doff + (size_t)i * np));
                J.ph.push_back(std::cos(arg));
                J.ph.push_back(std::sin(arg));
            }
            doff += (size_t)np * np;
        }
        J.D.assign(o->proj_rot, o->proj_rot + doff);
        for (double v : J.D)
            if (!std::isfinite(v)) return fail(RPA_ERR_INPUT, t + ": non-finite proj_rot entry");
        void* p = nullptr;
        int rc = get_buf(c, (B.prefix + "sym:P:" + tag).c_str(), 16 * (size_t)s->nbands * np_tot, B.s, &p);
        if (rc) return rc;
        J.P_in = static_cast<const double*>(s->P);
        J.P_out = static_cast<double*>(p);
        J.nproj = np_tot;
        d.P = p;
        up.add(J.tab, &J.d_tab);
        up.add(J.D, &J.d_D);
        up.add(J.ph, &J.d_ph);
    }
    B.usets.push_back(d);
    *out = &B.usets.back();
    return RPA_OK;
}

int enqueue_unfold(Batch& B) {
    for (const UnfoldJob& J : B.ujobs) {
        if (J.C_out) HIP_TRY(launch_conj_copy(J.C_in, J.nC, J.C_out, B.s));
        if (J.P_out)
            HIP_TRY(launch_rotate_proj(J.P_in, J.nb, J.nproj, static_cast<const int32_t*>(J.d_tab),
                                       static_cast<const double*>(J.d_D), static_cast<const double*>(J.d_ph), J.tr,
                                       J.P_out, B.s));
    }
    return RPA_OK;
}

int prepare_common(Batch& B, const rpa_states* k, Upload& up) {
    rpa_ctx* c = B.c;
    if (B.nw) {
        up.add(B.om, &B.d_om);
        up.add(B.ow, &B.d_ow);
    }
    for (int ax = 0; ax < 3; ++ax) {
        if (B.fp64()) {
            B.tw64[ax] = twiddles<double>(c->N[ax]);
            up.add(B.tw64[ax], &B.d_tw[ax]);
        } else {
            B.tw32[ax] = twiddles<float>(c->N[ax]);
            up.add(B.tw32[ax], &B.d_tw[ax]);
        }
    }
    const int na = k->natoms;
    B.poff.assign(na + 1, 0);
    B.qoff.assign(na + 1, 0);
    for (int a = 0; a <= na && na > 0; ++a) B.poff[a] = k->proj_off[a];
    for (int a = 0; a < na; ++a) {
        const int np = k->proj_off[a + 1] - k->proj_off[a];
        B.qoff[a + 1] = B.qoff[a] + np * np;
    }
    up.add(B.poff, &B.d_poff);
    up.add(B.qoff, &B.d_qoff);
    return RPA_OK;
}

int prepare_kset(Batch& B, KSet& K, Upload& up, const int32_t* pn_in = nullptr, const int32_t* pm_in = nullptr,
                 int np_in = -1) {
    const rpa_states* k = K.k;
    const rpa_states* kq = K.kq;
    if (np_in < 0) {
        pair_list(k, kq, K.pn, K.pm, B.m_major);
    } else {
        K.pn.assign(pn_in, pn_in + np_in);
        K.pm.assign(pm_in, pm_in + np_in);
        for (int i = 0; i < np_in; ++i)
            if (K.pn[i] < 0 || K.pn[i] >= k->nbands || K.pm[i] < 0 || K.pm[i] >= kq->nbands)
                return fail(RPA_ERR_SHAPE, "pair index out of range");
    }
    K.mapk = scatter_map(B.c, k);
    K.zcolk = grid_columns(B.c, K.mapk);
    up.add(K.pn, &K.d_pn);
    up.add(K.pm, &K.d_pm);
    up.add(K.mapk, &K.d_mapk);
    up.add(K.zcolk, &K.d_zcolk);
    if (!same_set(k, kq)) {
        K.mapkq = scatter_map(B.c, kq);
        K.zcolkq = grid_columns(B.c, K.mapkq);
        up.add(K.mapkq, &K.d_mapkq);
        up.add(K.zcolkq, &K.d_zcolkq);
    }
    K.epsk.assign(k->eps, k->eps + k->nbands);
    K.fk.assign(k->f, k->f + k->nbands);
    K.epskq.assign(kq->eps, kq->eps + kq->nbands);
    K.fkq.assign(kq->f, kq->f + kq->nbands);
    up.add(K.epsk, &K.d_epsk);
    up.add(K.fk, &K.d_fk);
    up.add(K.epskq, &K.d_epskq);
    up.add(K.fkq, &K.d_fkq);
    K.nlist_all.resize(k->nbands);
    std::iota(K.nlist_all.begin(), K.nlist_all.end(), 0);
    up.add(K.nlist_all, &K.d_nlist);
    K.drude_band.clear();
    K.drude_mdf.clear();
    if (k->dfde) {
        for (int n = 0; n < k->nbands; ++n)
            if (k->dfde[n] > 0.0) {
                K.drude_band.push_back(n);
                K.drude_mdf.push_back(k->dfde[n]);
            }
        if (!K.drude_band.empty()) {
            up.add(K.drude_band, &K.d_drude_band);
            up.add(K.drude_mdf, &K.d_drude_mdf);
        }
    }
    return RPA_OK;
}

int prepare_q(Batch& B, QJob& Q, Upload& up) {
    const QPlan& q = Q.qp;
    up.add(q.kx, &Q.d_kx);
    up.add(q.ky, &Q.d_ky);
    up.add(q.col_start, &Q.d_cs);
    up.add(q.col_g, &Q.d_cg);
    up.add(q.col_kz, &Q.d_ckz);
    up.add(q.zcol, &Q.d_zc);
    up.add(q.zcol_start, &Q.d_zcs);
    up.add(q.zcol_kz, &Q.d_zckz);
    up.add(q.vsqrt, &Q.d_vs);
    if (Q.qs->optical) {
        double qh[3] = {Q.qs->qhat[0], Q.qs->qhat[1], Q.qs->qhat[2]};
        const double nrm = std::sqrt(qh[0] * qh[0] + qh[1] * qh[1] + qh[2] * qh[2]);
        if (!(nrm > 0)) return fail(RPA_ERR_INPUT, "optical limit needs a nonzero qhat");
        for (int d = 0; d < 3; ++d) qh[d] /= nrm;
        Q.wq.resize(B.ks.size());
        Q.d_wq.assign(B.ks.size(), nullptr);
        for (size_t i = 0; i < B.ks.size(); ++i) {
            if (!Q.uses(i)) continue;
            const rpa_states* k = B.ks[i].k;
            Q.wq[i].resize(k->nQ);
            for (int j = 0; j < k->nQ; ++j) {
                double kv[3];
                kvec(B.c->B, k->kpt, k->miller + 3 * j, kv);
                Q.wq[i][j] = qh[0] * kv[0] + qh[1] * kv[1] + qh[2] * kv[2];
            }
            up.add(Q.wq[i], &Q.d_wq[i]);
        }
        const int nq2 = (int)B.qoff.back();
        Q.Dq.assign(std::max(nq2, 1), 0.0);
        for (int e = 0; e < nq2; ++e)
            Q.Dq[e] = qh[0] * Q.qs->Dpaw[e] + qh[1] * Q.qs->Dpaw[nq2 + e] + qh[2] * Q.qs->Dpaw[2 * nq2 + e];
        up.add(Q.Dq, &Q.d_Dq);
    }
    return RPA_OK;
}

void* buf(Batch& B, const char* name) { return (B.c->arena ? B.c->abufs : B.c->bufs)[B.prefix + name].p; }

// Work buffers, sized once for every q of the batch (never grown while launching).
struct WorkSizes {
    size_t tbuf = 0, rho = 0, weights = 0, paw_y = 0, paw_z = 0, pack = 0, scales = 0, chi = 0, drude = 0;
    size_t cholL = 0, cholP = 0, small = 0, phi_k = 0, phi_kq = 0;
};

int presize(Batch& B, bool need_ec, bool need_chi, WorkSizes& W) {
    rpa_ctx* c = B.c;
    const size_t vol = (size_t)c->N[0] * c->N[1] * c->N[2];
    const size_t el = B.elem();
    // bytes of the MFMA PAW term's Z buffer at most
    size_t paw_zcap = (size_t)2 << 30;
    if (c->cap) paw_zcap = std::min(paw_zcap, c->cap / 8);
    if (c->arena) paw_zcap = std::min(paw_zcap, c->arena_cap / 8);
    B.paw_mwin = 0;
    // bands n and m the pairs of each k set span (the choice of the PAW term's form does not depend on
    // the chunking, so that a pair's density does not either)
    int nspan_max = 0, mspan_max = 0;
    for (auto& K : B.ks) {
        if (K.pn.empty()) continue;
        const auto n = std::minmax_element(K.pn.begin(), K.pn.end());
        const auto m = std::minmax_element(K.pm.begin(), K.pm.end());
        nspan_max = std::max(nspan_max, *n.second - *n.first + 1);
        mspan_max = std::max(mspan_max, *m.second - *m.first + 1);
    }
    for (auto& K : B.ks) {
        W.drude += K.drude_band.size() * sizeof(double);
        W.phi_k = std::max(W.phi_k, (size_t)K.k->nbands * vol * 2 * el);
        if (!same_set(K.k, K.kq)) W.phi_kq = std::max(W.phi_kq, (size_t)K.kq->nbands * vol * 2 * el);
    }
    int P = 0;
    for (auto& K : B.ks) P = std::max(P, (int)K.pn.size());
    // rank-k variant (new size buckets autotuned first) and pair chunk of every q-point; with a shared pair
    // transform every q-point takes the smallest chunk
    for (auto& Q : B.qj) {
        const PairGeom& g = Q.qp.g;
        if (!B.fp64() && c->autotune && !c->arena && !c->capturing && P > 0 &&
            !c->tune.count(tune_key(B.prec, g.NGp))) {
            // the first call with a sphere of this size bucket times the rank-k variants on it
            const int b = tune_bucket(g.NGp);
            if (!c->tune.count(tune_key(B.prec, b))) {
                int rc = autotune_run(c, B.prec, b, std::max(256, std::min(P, 8192)), B.nw, B.s);
                if (rc) return rc;
            }
            c->tune[tune_key(B.prec, g.NGp)] = c->tune[tune_key(B.prec, b)];
        }
        Q.variant = default_variant(c, B.prec, g.NGp);
        Q.Pc = std::max(1, std::min(P, chunk_size(c, Q.qp, B.nw, el, Q.variant)));
    }
    if (B.share_xy) {
        int pc = B.qj.empty() ? 1 : B.qj[0].Pc;
        for (auto& Q : B.qj) pc = std::min(pc, Q.Pc);
        for (auto& Q : B.qj) Q.Pc = pc;
    }
    for (auto& Q : B.qj) {
        const PairGeom& g = Q.qp.g;
        const int Pc = Q.Pc;
        const int nproj = B.poff.empty() ? 0 : B.poff.back();
        // band windows of a chunk: n (factorised VALU PAW term) and m (MFMA PAW term)
        int win = 1, mspan = 1;
        for (auto& K : B.ks) {
            for (size_t p0 = 0; p0 < K.pn.size(); p0 += Pc) {
                const size_t p1 = std::min(K.pn.size(), p0 + Pc);
                int lo = K.pn[p0], hi = K.pn[p0], mlo = K.pm[p0], mhi = K.pm[p0];
                for (size_t i = p0; i < p1; ++i) {
                    lo = std::min(lo, (int)K.pn[i]);
                    hi = std::max(hi, (int)K.pn[i]);
                    mlo = std::min(mlo, (int)K.pm[i]);
                    mhi = std::max(mhi, (int)K.pm[i]);
                }
                win = std::max(win, hi - lo + 1);
                mspan = std::max(mspan, mhi - mlo + 1);
            }
        }

        W.tbuf = std::max(W.tbuf, (size_t)Pc * g.N3 * g.ncols * 2 * el);
        W.rho = std::max(W.rho, 2 * (size_t)Pc * g.NGp * el);
        const int lda = (Pc + 3) / 4 * 4;
        W.weights = std::max(W.weights, (size_t)std::max(B.nw, 1) * lda * sizeof(double));
        if (nproj > 0) {
            W.paw_y = std::max(W.paw_y, 2 * (size_t)win * nproj * g.NGp * el);
            // Z of at most paw_zcap bytes: a chunk whose pairs span more bands m runs the MFMA PAW term over
            // windows of consecutive pairs with fewer bands
            const size_t per_m = 2 * (size_t)nproj * g.NGp * el;
            int mwin = (int)std::max<size_t>(1, std::min<size_t>((size_t)mspan, paw_zcap / per_m));
            if (c->paw_win > 0) mwin = std::min(mwin, c->paw_win);
            B.paw_mwin = B.paw_mwin ? std::min(B.paw_mwin, mwin) : mwin;
        }
        if (!B.fp64()) {
            const int NGq = (g.NGp + 127) / 128 * 128;
            const size_t blk = (size_t)((Pc + 31) / 32) * NGq * 32;
            W.pack = std::max(W.pack, blk * (2 * sizeof(float) + 4 * sizeof(unsigned short)));
            W.scales = std::max(W.scales, (size_t)(B.nw + 1 + 256) * sizeof(float));
        }
        B.ld = std::max(B.ld, Q.ld);
    }
    // the MFMA PAW term factorised per band n (Y_n for the bands n of a chunk) where the pairs span fewer
    // bands n than bands m and Y fits, else per band m (Z_m for the bands of a window, at most paw_mwin of them);
    // the factorised VALU form (Y for every band n) serves the adjoint
    if (B.paw_mwin > 0)
        for (auto& Q : B.qj) {
            const int nproj = B.poff.empty() ? 0 : B.poff.back();
            W.paw_z = std::max(W.paw_z, 2 * (size_t)B.paw_mwin * nproj * Q.qp.g.NGp * el);
        }
    B.paw_mfma = B.allow_paw_mfma && W.paw_z > 0;
    B.paw_nform = B.paw_mfma && c->paw_win == 0 && nspan_max <= mspan_max && W.paw_y <= paw_zcap;
    if (B.paw_nform) W.paw_z = 0;
    else if (B.paw_mfma) W.paw_y = 0;
    else W.paw_z = 0;
    // per class of q-points with one leading dimension: all real parts, then all imaginary parts, so that
    // matrix b = (q - q0) nw + w of the class sits at b * ld^2 and the E_c stage factorises the class as
    // one set of matrices
    const size_t nmat = B.qj.size() * (size_t)B.nw;
    size_t chi_doubles = 0, cls_mat_max = 0, panel_max = 0;
    for (auto& C : B.cls) {
        const size_t cm = (size_t)C.nq * B.nw;
        chi_doubles += 2 * cm * (size_t)C.ld * C.ld;
        cls_mat_max = std::max(cls_mat_max, cm);
        panel_max = std::max(panel_max, cm * (size_t)C.ld);
    }
    if (need_ec || need_chi) W.chi = chi_doubles * sizeof(double);
    if (need_ec) {
        W.cholL = 2 * cls_mat_max * kTile * kTile * sizeof(double);
        W.cholP = 2 * 2 * panel_max * 2 * kTile * sizeof(double);   // two pairs of panels in flight
        W.small = nmat * (2 * sizeof(double) + sizeof(int)) + 64;
    }
    struct NB {
        const char* n;
        size_t b;
    } list[] = {{"phi_k", W.phi_k}, {"phi_kq", W.phi_kq}, {"tbuf", W.tbuf}, {"rho", W.rho},
                {"weights", W.weights}, {"paw_y", W.paw_y}, {"paw_z", W.paw_z}, {"drude", W.drude},
                {"split_pack", W.pack},
                {"split_scales", W.scales},
                {"chi", W.chi}, {"chol_L", W.cholL}, {"chol_panel", W.cholP}, {"ec_small", W.small}};
    for (auto& e : list) {
        if (!e.b) continue;
        void* p = nullptr;
        int rc = get_buf(c, (B.prefix + e.n).c_str(), e.b, B.s, &p);
        if (rc) return rc;
    }
    if (W.chi) {
        double* base = static_cast<double*>(buf(B, "chi"));
        for (auto& C : B.cls) {
            const size_t l2 = (size_t)C.ld * C.ld, cm = (size_t)C.nq * B.nw;
            C.cr = base;
            C.ci = base + cm * l2;
            for (int i = 0; i < C.nq; ++i) {
                B.qj[C.q0 + i].cr = C.cr + (size_t)i * B.nw * l2;
                B.qj[C.q0 + i].ci = C.ci + (size_t)i * B.nw * l2;
            }
            base += 2 * cm * l2;
        }
    }
    return RPA_OK;
}

template <typename T>
int enqueue_orbitals(Batch& B, const rpa_states* s, void* d_map, const std::vector<int32_t>& zcols, void* d_zcols,
                     const char* name, cplx<T>** out) {
    rpa_ctx* c = B.c;
    const size_t vol = (size_t)c->N[0] * c->N[1] * c->N[2];
    cplx<T>* phi = static_cast<cplx<T>*>(buf(B, name));
    ProfScope ps_(c, S_ORB, B.s);
    HIP_TRY(launch_fill_zero<T>(phi, (size_t)s->nbands * vol, B.s));
    HIP_TRY(launch_orb_scatter<T>(static_cast<const double*>(s->C), s->nbands, s->nQ,
                                  static_cast<const int32_t*>(d_map), vol, phi, B.s));
    // z, then x and y: register-resident lines where the axis length has them, LDS passes otherwise
    // (only the columns that hold coefficients: the rest of the grid is zero and stays so along z)
    hipError_t e = c->pair_reg ? launch_grid_fft_z_reg<T>(phi, s->nbands, c->N[0], c->N[1], c->N[2], +1,
                                                          static_cast<const int32_t*>(d_zcols), (int)zcols.size(),
                                                          B.s)
                               : hipErrorNotSupported;
    if (e == hipErrorNotSupported)
        HIP_TRY(launch_fft_axis<T>(phi, s->nbands, c->N[0], c->N[1], c->N[2], 2, c->plan[2],
                                   static_cast<const cplx<T>*>(B.d_tw[2]), +1, B.s));
    else
        HIP_TRY(e);
    e = c->pair_reg ? launch_grid_fft_xy_reg<T>(phi, s->nbands, c->N[0], c->N[1], c->N[2], +1, B.s)
                    : hipErrorNotSupported;
    if (e == hipErrorNotSupported) {
        for (int ax = 0; ax < 2; ++ax)
            HIP_TRY(launch_fft_axis<T>(phi, s->nbands, c->N[0], c->N[1], c->N[2], ax, c->plan[ax],
                                       static_cast<const cplx<T>*>(B.d_tw[ax]), +1, B.s));
    } else {
        HIP_TRY(e);
    }
    *out = phi;
    return RPA_OK;
}

// rho for pairs [p0, p0 + np) of K into planar buffers rre/rim [np][NGp]
template <typename T>
// skip_xy: the chunk's x-y transform is already in tbuf (computed for another q-point of the same box)
int enqueue_pairs(Batch& B, QJob& Q, KSet& K, int ik, const cplx<T>* phik, const cplx<T>* phikq, int p0, int np,
                  T* rre, T* rim, bool skip_xy = false) {
    rpa_ctx* c = B.c;
    const PairGeom& g = Q.qp.g;
    cplx<T>* tb = static_cast<cplx<T>*>(buf(B, "tbuf"));
    const int32_t* pn = static_cast<const int32_t*>(K.d_pn) + p0;
    const int32_t* pm = static_cast<const int32_t*>(K.d_pm) + p0;
    const bool reg_xy = c->pair_reg && pair_xy_reg_supported<T>(g);
    const bool reg_z = c->pair_reg && pair_z_reg_supported<T>(g);
    const bool quad_z = c->pair_reg && !reg_z && pair_z_quad_supported<T>(g);
    if (!skip_xy) {
        ProfScope ps_(c, S_PAIR_XY, B.s);
        if (reg_xy)
            HIP_TRY(launch_pair_xy_reg<T>(phik, phikq, pn, pm, np, g, tb, B.s));
        else
            HIP_TRY(launch_pair_xy<T>(phik, phikq, pn, pm, np, g, static_cast<const int32_t*>(Q.d_kx),
                                      static_cast<const int32_t*>(Q.d_ky), static_cast<const cplx<T>*>(B.d_tw[0]),
                                      static_cast<const cplx<T>*>(B.d_tw[1]), tb, B.s));
    }
    {
        ProfScope ps_(c, S_PAIR_Z, B.s);
        if (reg_z)
            HIP_TRY(launch_pair_z_reg<T>(tb, np, g, static_cast<const int32_t*>(Q.d_zc),
                                         static_cast<const int32_t*>(Q.d_zcs), static_cast<const int32_t*>(Q.d_cg),
                                         static_cast<const int32_t*>(Q.d_zckz), rre, rim, B.s));
        else if (quad_z)
            HIP_TRY(launch_pair_z_quad<T>(tb, np, g, static_cast<const int32_t*>(Q.d_zc),
                                          static_cast<const int32_t*>(Q.d_zcs), static_cast<const int32_t*>(Q.d_cg),
                                          static_cast<const int32_t*>(Q.d_zckz), rre, rim, B.s));
        else
            HIP_TRY(launch_pair_z_gather<T>(tb, np, g, static_cast<const int32_t*>(Q.d_zc),
                                            static_cast<const int32_t*>(Q.d_zcs), static_cast<const int32_t*>(Q.d_cg),
                                            static_cast<const int32_t*>(Q.d_zckz),
                                            static_cast<const cplx<T>*>(B.d_tw[2]), rre, rim, B.s));
    }
    const int nproj = nproj_total(K.k);
    if (nproj > 0 && B.paw_nform) {
        // Y_n for the chunk's bands n, then the GEMM over the chunk's pairs grouped by n
        const auto it = B.pawn.find(std::make_pair(ik, Q.Pc));
        const int ci = p0 / Q.Pc;
        if (it == B.pawn.end() || ci >= (int)it->second.s0.size() || p0 % Q.Pc)
            return fail(RPA_ERR_SHAPE, "PAW pair tables missing for a chunk");
        const PawN& PT = it->second;
        const int nlo = PT.nlo[ci], nn = PT.nn[ci];
        T* Yre = static_cast<T*>(buf(B, "paw_y"));
        T* Yim = Yre + (size_t)nn * nproj * g.NGp;
        ProfScope ps_(c, S_PAW, B.s);
        HIP_TRY(launch_paw_yn<T>(static_cast<const double*>(K.k->P), nproj, nlo, nn,
                                 static_cast<const int32_t*>(B.d_poff), static_cast<const int32_t*>(B.d_qoff),
                                 K.k->natoms, nproj, static_cast<const double*>(Q.qs->Qpaw), g.NG, g.NGp, Yre, Yim,
                                 B.s));
        HIP_TRY(launch_paw_mfma_n<T>(Yre, Yim, nproj, static_cast<const double*>(K.kq->P), nproj, pm,
                                     static_cast<const int32_t*>(PT.d_seg) + 3 * (size_t)PT.s0[ci], PT.ns[ci],
                                     static_cast<const int32_t*>(PT.d_perm) + p0, g.NGp, rre, rim, B.s));
    } else if (nproj > 0 && B.paw_mfma) {
        // windows of consecutive pairs whose bands m span at most paw_mwin (one window per chunk unless the
        // chunk's pairs span more bands than the Z buffer holds)
        T* Zr = static_cast<T*>(buf(B, "paw_z"));
        ProfScope ps_(c, S_PAW, B.s);
        for (int a = 0; a < np;) {
            int mlo = K.pm[p0 + a], mhi = mlo, b = a + 1;
            for (; b < np; ++b) {
                const int m = K.pm[p0 + b];
                const int lo = std::min(mlo, m), hi = std::max(mhi, m);
                if (hi - lo + 1 > B.paw_mwin) break;
                mlo = lo;
                mhi = hi;
            }
            const int nm = mhi - mlo + 1;
            T* Zi = Zr + (size_t)nm * nproj * g.NGp;
            HIP_TRY(launch_paw_mfma<T>(static_cast<const double*>(K.k->P), static_cast<const double*>(K.kq->P), nproj,
                                       pn + a, pm + a, b - a, mlo, nm, static_cast<const int32_t*>(B.d_poff),
                                       static_cast<const int32_t*>(B.d_qoff), K.k->natoms, nproj,
                                       static_cast<const double*>(Q.qs->Qpaw), g.NG, g.NGp, Zr, Zi,
                                       rre + (size_t)a * g.NGp, rim + (size_t)a * g.NGp, B.s));
            a = b;
        }
    } else if (nproj > 0) {
        int nlo = K.pn[p0], nhi = K.pn[p0];
        for (int i = p0; i < p0 + np; ++i) {
            nlo = std::min(nlo, (int)K.pn[i]);
            nhi = std::max(nhi, (int)K.pn[i]);
        }
        const int nn = nhi - nlo + 1;
        T* Yre = static_cast<T*>(buf(B, "paw_y"));
        T* Yim = Yre + (size_t)nn * nproj * g.NGp;
        ProfScope ps_(c, S_PAW, B.s);
        HIP_TRY(launch_paw_y<T>(static_cast<const double*>(K.k->P), nproj, static_cast<const int32_t*>(K.d_nlist) + nlo,
                                nn, static_cast<const int32_t*>(B.d_poff), static_cast<const int32_t*>(B.d_qoff),
                                K.k->natoms, nproj, static_cast<const double*>(Q.qs->Qpaw), g.NG, g.NGp, Yre, Yim,
                                B.s));
        HIP_TRY(launch_paw_add<T>(Yre, Yim, pn, nlo, pm, static_cast<const double*>(K.kq->P), nproj, nproj, np, g.NG,
                                  g.NGp, rre, rim, B.s));
    }
    if (Q.qs->optical && Q.qp.g0 >= 0) {
        ProfScope ps_(c, S_OPTICAL, B.s);
        HIP_TRY(launch_optical_row<T>(static_cast<const double*>(K.k->C), static_cast<const double*>(K.kq->C), K.k->nQ,
                                      static_cast<const double*>(Q.d_wq[ik]), static_cast<const double*>(K.k->P),
                                      static_cast<const double*>(K.kq->P), nproj, static_cast<const double*>(Q.d_Dq),
                                      static_cast<const int32_t*>(B.d_poff), static_cast<const int32_t*>(B.d_qoff),
                                      K.k->natoms, static_cast<const double*>(K.d_epsk),
                                      static_cast<const double*>(K.d_epskq), pn, pm, np, Q.qp.g0, g.NGp, rre, rim,
                                      B.s));
    }
    return RPA_OK;
}

// chi0(w) += rho diag(a(w)) rho^H for one chunk, with the job's kernel variant
// chi0 accumulator of one job: nw matrices of ld x ld, real and imaginary blocks
hipError_t zero_accumulator(Batch& B, QJob& Q) {
    const size_t n = (size_t)B.nw * Q.ld * Q.ld / 2;   // complex pairs of doubles per block
    hipError_t e = launch_fill_zero<double>(reinterpret_cast<cplx<double>*>(Q.cr), n, B.s);
    if (e != hipSuccess) return e;
    return launch_fill_zero<double>(reinterpret_cast<cplx<double>*>(Q.ci), n, B.s);
}

template <typename T>
int enqueue_update(Batch& B, QJob& Q, int np, const T* rre, const T* rim, const double* aw, int lda) {
    rpa_ctx* c = B.c;
    const int NGp = Q.qp.NGp;
    // the first update of an accumulator: variants 4 and 5 store instead of adding (their tiles cover the
    // lower triangle of this q-point's padded sphere, which is all the chi0 output reads; the E_c stage
    // assigns zero to the rest of a batch's common leading dimension); variant 1 adds into a zero-filled
    // accumulator
    const bool store_first = Q.fresh && sizeof(T) == 4 && Q.variant >= 4;
    if (Q.fresh && !store_first) HIP_TRY(zero_accumulator(B, Q));
    Q.fresh = false;
    if constexpr (sizeof(T) == 8) {
        ProfScope ps_(c, S_HERK, B.s);
        HerkArgs h{};
        h.Are = reinterpret_cast<const double*>(rre);
        h.Aim = reinterpret_cast<const double*>(rim);
        h.sA = 0;
        h.ldA = NGp;
        h.colA = 0;
        h.K = np;
        h.w = aw;
        h.sw = lda;
        h.alpha = 0;
        h.Cre = Q.cr;
        h.Cim = Q.ci;
        h.sC = (long long)Q.ld * Q.ld;
        h.ldC = Q.ld;
        h.r0 = 0;
        h.nT = NGp / kTile;
        h.nbatch = B.nw;
        HIP_TRY(launch_herk_f64(h, B.s));
    } else {
        const bool fp16 = B.prec == RPA_SPLIT_FP16;
        float* scales = nullptr;
        // operands of the pipelined kernels: the FP32 pair densities in K-steps of 32 pairs and the
        // pre-split 16-bit hi/lo of each
        const int NGq = (NGp + 127) / 128 * 128;
        const size_t blk = (size_t)((np + 31) / 32) * NGq * 32;
        float* Xre = nullptr;
        float* Xim = nullptr;
        unsigned short* Bp[4] = {nullptr, nullptr, nullptr, nullptr};
        {
            ProfScope pp_(c, S_PACK, B.s);
            if (fp16) {
                scales = static_cast<float*>(buf(B, "split_scales"));
                HIP_TRY(launch_split_scales(reinterpret_cast<const float*>(rre), reinterpret_cast<const float*>(rim),
                                            (size_t)np * NGp, aw, lda, np, B.nw, scales, scales + B.nw + 1, B.s));
            }
            if (Q.variant >= 2) {
                Xre = static_cast<float*>(buf(B, "split_pack"));
                Xim = Xre + blk;
                for (int q = 0; q < 4; ++q) Bp[q] = reinterpret_cast<unsigned short*>(Xim + blk) + q * blk;
                HIP_TRY(launch_pack_split(reinterpret_cast<const float*>(rre), reinterpret_cast<const float*>(rim),
                                          np, NGp, NGq, scales, B.nw, fp16, Xre, Xim, Bp, B.s));
            }
        }
        ProfScope ps_(c, S_HERK, B.s);
        if (Q.variant >= 2) {
            HerkSplit2Args h{};
            h.Xre = Xre;
            h.Xim = Xim;
            for (int q = 0; q < 4; ++q) h.B[q] = Bp[q];
            h.NGq = NGq;
            h.K = np;
            h.w = aw;
            h.lda = lda;
            h.Cre = Q.cr;
            h.Cim = Q.ci;
            h.sC = (long long)Q.ld * Q.ld;
            h.ldC = Q.ld;
            h.nw = B.nw;
            h.fp16 = fp16;
            h.scales = scales;
            h.overwrite = store_first;
            // 64-row blocks I of the lower triangle, each with column blocks 0 .. I/2 of 128
            const int nR = NGp / kTile;
            h.ntiles = 0;
            for (int I = 0; I < nR; ++I) h.ntiles += I / 2 + 1;
            HIP_TRY(launch_herk_split4(h, Q.variant == 5, B.s));
        } else {
            HerkSplitArgs h{};
            h.Are = reinterpret_cast<const float*>(rre);
            h.Aim = reinterpret_cast<const float*>(rim);
            h.ldA = NGp;
            h.K = np;
            h.w = aw;
            h.lda = lda;
            h.Cre = Q.cr;
            h.Cim = Q.ci;
            h.sC = (long long)Q.ld * Q.ld;
            h.ldC = Q.ld;
            h.nT = NGp / kTile;
            h.nw = B.nw;
            h.fp16 = fp16;
            h.wscale = scales;
            HIP_TRY(launch_herk_split(h, B.s));
        }
    }
    return RPA_OK;
}

// chi0 of every q of the batch (planar lower tiles in each job's accumulator)
template <typename T>
int enqueue_chi0(Batch& B) {
    rpa_ctx* c = B.c;
    int urc = enqueue_unfold(B);
    if (urc) return urc;
    // every accumulator starts fresh: its first update stores or zero-fills it (one with no update at all
    // is zero-filled at the end)
    for (auto& Q : B.qj) Q.fresh = true;
    for (size_t ik = 0; ik < B.ks.size(); ++ik) {
        KSet& K = B.ks[ik];
        const int P = (int)K.pn.size();
        if (P == 0) continue;
        cplx<T>* phik = nullptr;
        cplx<T>* phikq = nullptr;
        int rc = enqueue_orbitals<T>(B, K.k, K.d_mapk, K.zcolk, K.d_zcolk, "phi_k", &phik);
        if (rc) return rc;
        if (same_set(K.k, K.kq)) {
            phikq = phik;
        } else {
            rc = enqueue_orbitals<T>(B, K.kq, K.d_mapkq, K.zcolkq, K.d_zcolkq, "phi_kq", &phikq);
            if (rc) return rc;
        }
        const double prefac = K.k->weight / c->volume;
        // one chunk of one q-point: pair densities (the x-y transform skipped when shared), weights, update
        auto chunk = [&](QJob& Q, int p0, int np, bool skip_xy) -> int {
            const int Pc = Q.Pc;
            const int lda = (Pc + 3) / 4 * 4;
            T* rre = static_cast<T*>(buf(B, "rho"));
            T* rim = rre + (size_t)Pc * Q.qp.NGp;
            double* aw = static_cast<double*>(buf(B, "weights"));
            int r = enqueue_pairs<T>(B, Q, K, (int)ik, phik, phikq, p0, np, rre, rim, skip_xy);
            if (r) return r;
            {
                ProfScope ps_(c, S_WEIGHTS, B.s);
                if (B.realfreq)
                    HIP_TRY(launch_weights_real(
                        static_cast<const double*>(K.d_epsk), static_cast<const double*>(K.d_epskq),
                        static_cast<const double*>(K.d_fk), static_cast<const double*>(K.d_fkq),
                        static_cast<const int32_t*>(K.d_pn) + p0, static_cast<const int32_t*>(K.d_pm) + p0, np,
                        static_cast<const double*>(B.d_om), B.nw_user, B.eta, prefac, aw, lda, B.s));
                else
                    HIP_TRY(launch_weights(static_cast<const double*>(K.d_epsk),
                                           static_cast<const double*>(K.d_epskq),
                                           static_cast<const double*>(K.d_fk), static_cast<const double*>(K.d_fkq),
                                           static_cast<const int32_t*>(K.d_pn) + p0,
                                           static_cast<const int32_t*>(K.d_pm) + p0, np,
                                           static_cast<const double*>(B.d_om), B.nw, prefac, aw, lda, B.s));
            }
            return enqueue_update<T>(B, Q, np, rre, rim, aw, lda);
        };
        if (B.share_xy) {
            // chunk by chunk: the x-y transform once (with the first q-point), then every q-point's sphere
            const int Pc = B.qj[0].Pc;
            for (int p0 = 0; p0 < P; p0 += Pc) {
                const int np = std::min(Pc, P - p0);
                for (size_t j = 0; j < B.qj.size(); ++j) {
                    rc = chunk(B.qj[j], p0, np, j > 0);
                    if (rc) return rc;
                }
            }
        } else {
            for (auto& Q : B.qj) {
                if (!Q.uses(ik)) continue;
                for (int p0 = 0; p0 < P; p0 += Q.Pc) {
                    rc = chunk(Q, p0, std::min(Q.Pc, P - p0), false);
                    if (rc) return rc;
                }
            }
        }
    }
    for (auto& Q : B.qj)
        if (Q.fresh) HIP_TRY(zero_accumulator(B, Q));
    // intraband head of the optical q-points (sets that carry -df/de): term per band, then the head of every
    // frequency's accumulator
    for (auto& Q : B.qj) {
        if (!Q.qs->optical || Q.qp.g0 < 0) continue;
        double* term = static_cast<double*>(buf(B, "drude"));
        int nt = 0;
        for (size_t ik = 0; ik < B.ks.size(); ++ik) {
            KSet& K = B.ks[ik];
            if (K.drude_band.empty() || !Q.uses(ik)) continue;
            ProfScope ps_(c, S_OPTICAL, B.s);
            HIP_TRY(launch_band_drude(static_cast<const double*>(K.k->C), K.k->nQ, static_cast<const double*>(Q.d_wq[ik]),
                                      static_cast<const double*>(K.k->P), nproj_total(K.k),
                                      static_cast<const double*>(Q.d_Dq), static_cast<const int32_t*>(B.d_poff),
                                      static_cast<const int32_t*>(B.d_qoff), K.k->natoms,
                                      static_cast<const int32_t*>(K.d_drude_band),
                                      static_cast<const double*>(K.d_drude_mdf), (int)K.drude_band.size(),
                                      K.k->weight, term + nt, B.s));
            nt += (int)K.drude_band.size();
        }
        if (nt > 0 && B.realfreq)
            HIP_TRY(launch_add_drude_real(term, nt, static_cast<const double*>(B.d_om), B.nw_user, B.eta,
                                          1.0 / c->volume, Q.cr + (size_t)Q.qp.g0 * Q.ld + Q.qp.g0,
                                          (long long)Q.ld * Q.ld, B.s));
        else if (nt > 0)
            HIP_TRY(launch_add_drude(term, nt, static_cast<const double*>(B.d_om), B.nw, 1.0 / c->volume,
                                     Q.cr + (size_t)Q.qp.g0 * Q.ld + Q.qp.g0, (long long)Q.ld * Q.ld, B.s));
    }
    return RPA_OK;
}

// side stream and events of the Cholesky look-ahead (created outside any graph capture)
int ensure_lookahead(rpa_ctx* c) {
    if (!c->la_stream) HIP_TRY(hipStreamCreateWithFlags(&c->la_stream, hipStreamNonBlocking));
    if (!c->la2_stream) HIP_TRY(hipStreamCreateWithFlags(&c->la2_stream, hipStreamNonBlocking));
    for (auto& e : c->la_ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : c->la2_ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return RPA_OK;
}

// E_c of every job of the batch from its accumulator (overwritten by -K and its
// factor). The nq * nw matrices share one leading dimension and are factorised
// together, so each 64-column panel step is one launch for the whole batch.
// from_full (one job): -K from a caller chi0 [nw][NG][NG] instead.
// Lblocks (one job): keep every inverted diagonal block and the factor itself.
//
// Blocking and look-ahead. The panel steps go in pairs (j = 2p, 2p+1) and the trailing matrix is
// updated once per pair, with K = 128 (both solved panels of the pair): half the passes over the
// trailing matrix of an update per step. The solved panels of pair p share one buffer of two
// 64-row slots, and the pairs alternate between two such buffers.
//   even step j: panel, solve into slot 0, then a_j: block column j+1 with P_j (K = 64);
//   odd step j:  panel, solve into slot 1, then b_p on la_stream: every block column from j+3 on
//                with K = 128, and a'_p: block columns j+1 and j+2 with K = 128, after b_{p-1}
//                (which covers them), on the main stream.
// b_p covers none of the block columns the next pair's panels need before a'_p has run, so the b's
// run back to back on la_stream while the main stream factors the next pair; b_p starts after a'_p's
// diagonal tile, so that this tile is not queued behind the whole update. Every look-ahead update
// (a_j, a'_p) runs the diagonal tile of its first block column on the main stream, where the next
// panel reads it, and the rest on la2_stream beside that panel: first the rows below that tile, which
// the next solve waits for, then (a'_p) the second block column, which the next look-ahead's diagonal
// tile waits for. Ordering of the updates that touch the same tiles: b_{p-1} before a'_p (main stream
// wait); a'_p's second block column before a_{j+1} (the main stream's wait before a_{j+1}'s diagonal
// tile, and la2_stream order for its rest); every rest before the solve that reads its block column.
// A pair buffer is overwritten by the solves of pair p+2, after the main stream has waited for b_p
// (at a'_{p+1}) and for the rests on la2_stream.
int enqueue_ec_class(Batch& B, const QClass& C, bool from_full, const void* chi_full, double* Lblocks) {
    rpa_ctx* c = B.c;
    const int nw = B.nw, ld = C.ld;
    const int nq = C.nq, q0 = C.q0;
    const int nb = nq * nw;
    // per-matrix scalars of the whole batch: ln det [all], Tr K [all], failure flags [all]; this class's
    // matrices are entries q0 nw .. (q0 + nq) nw - 1
    const int nbt = (int)B.qj.size() * nw;
    double* logdet = static_cast<double*>(buf(B, "ec_small")) + (size_t)q0 * nw;
    double* trk = logdet + nbt;
    int* failv = reinterpret_cast<int*>(static_cast<double*>(buf(B, "ec_small")) + 2 * (size_t)nbt) + (size_t)q0 * nw;
    double* Lre = static_cast<double*>(buf(B, "chol_L"));
    double* Lim = Lre + (size_t)nb * kTile * kTile;
    double* Pbase = static_cast<double*>(buf(B, "chol_panel"));
    // pair buffers: [2][re, im][nb][2 * kTile][ld]
    const size_t pslot = (size_t)kTile * ld;   // one slot of one matrix
    const size_t pmat = 2 * pslot;             // both slots of one matrix (the matrix stride)
    const size_t ppart = (size_t)nb * pmat;    // the real (or imaginary) part of a pair buffer
    double* cr = C.cr;
    double* ci = C.ci;
    const long long ld2 = (long long)ld * ld;
    int rc = ensure_lookahead(c);
    if (rc) return rc;
    hipStream_t M = B.s, S = c->la_stream, S2 = c->la2_stream;
    hipEvent_t evA = c->la_ev[0], evD = c->la2_ev[0], evR = c->la2_ev[1], evR2 = c->la2_ev[2];
    ProfScope ps_(c, S_CHOL, M);
    HIP_TRY(launch_zero(logdet, nb, failv, nb, M));
    for (int qi = 0; qi < nq; ++qi) {
        QJob& Q = B.qj[q0 + qi];
        if (from_full) {
            HIP_TRY(launch_build_negk_from_full(static_cast<const double*>(chi_full), Q.qp.NG, Q.cr, Q.ci, ld, nw,
                                                static_cast<const double*>(Q.d_vs), trk + qi * nw, M));
        } else {
            HIP_TRY(launch_build_negk(Q.cr, Q.ci, ld, Q.qp.NG, ld, nw, static_cast<const double*>(Q.d_vs),
                                      trk + qi * nw, M));
        }
    }
    // C[rows r, columns c] -= sum_k P[k][r] conj(P[k][c]) for k < K from the panel buffer at P
    auto lookahead = [&](double* Pr, double* Pi, int K, int r, int col, int rows, int cols, int lower,
                         hipStream_t st) -> hipError_t {
        GemmArgs g{};
        g.M = rows;
        g.N = cols;
        g.K = K;
        g.nbatch = nb;
        g.Ar = Pr + r;
        g.Ai = Pi + r;
        g.sA = (long long)pmat;
        g.aI = 1;
        g.aK = ld;
        g.conjA = 0;
        g.Br = Pr + col;
        g.Bi = Pi + col;
        g.sB = (long long)pmat;
        g.bK = ld;
        g.bJ = 1;
        g.conjB = 1;
        g.Cr = cr + (size_t)r * ld + col;
        g.Ci = ci + (size_t)r * ld + col;
        g.sC = ld2;
        g.ldC = ld;
        g.alpha = -1.0;
        g.beta = 1;
        g.lower = lower;
        return lower ? launch_gemm_c64_shortk(g, st) : launch_gemm_c64(g, st);
    };
    bool pending_b = false;   // a pair's trailing update is in flight on S
    int last_p = 0;           // pair of the last one
    bool pending_r = false;   // the rest of a look-ahead update's first block column is in flight on S2
    bool pending_r2 = false;  // and that of its second block column (K = 128 look-aheads)
    for (int j0 = 0; j0 < ld; j0 += kTile) {
        const int step = j0 / kTile, pair = step >> 1, slot = step & 1;
        double* PPre = Pbase + (size_t)(pair & 1) * 2 * ppart;   // this pair's buffer
        double* PPim = PPre + ppart;
        double* Pre = PPre + slot * pslot;                       // this step's slot
        double* Pim = PPim + slot * pslot;
        if (Lblocks) {
            // keep every inverted diagonal block: [block][re/im][w][64][64]
            Lre = Lblocks + (size_t)step * 2 * nb * kTile * kTile;
            Lim = Lre + (size_t)nb * kTile * kTile;
        }
        // panel j: the diagonal tile of block column j is complete (its look-ahead tile ran before it
        // here, and every trailing update that covers it was waited for before that)
        HIP_TRY(launch_chol_panel(cr, ci, ld, j0, nb, Lre, Lim, logdet, failv, M));
        const int r0 = j0 + kTile;
        if (r0 >= ld) break;
        // the rows below the diagonal tile are complete once the rest of the last look-ahead is
        if (pending_r) HIP_TRY(hipStreamWaitEvent(M, evR, 0));
        pending_r = false;
        if (Lblocks) {
            // the adjoint needs the factor itself: L21 also replaces the block column
            HIP_TRY(launch_chol_trsm(cr, ci, ld, j0, ld, nb, Lre, Lim, Pre, Pim, (long long)pmat, M));
        } else {
            // panel operand of the updates only: P[c][r] = sum_k conj(L11^-1[c][k]) A21[r][k]
            GemmArgs gm{};
            gm.M = kTile;
            gm.N = ld - r0;
            gm.K = kTile;
            gm.nbatch = nb;
            gm.Ar = Lre;
            gm.Ai = Lim;
            gm.sA = (long long)kTile * kTile;
            gm.aI = kTile;
            gm.aK = 1;
            gm.conjA = 1;
            gm.Br = cr + (size_t)r0 * ld + j0;
            gm.Bi = ci + (size_t)r0 * ld + j0;
            gm.sB = ld2;
            gm.bK = 1;
            gm.bJ = ld;
            gm.conjB = 0;
            gm.Cr = Pre + r0;
            gm.Ci = Pim + r0;
            gm.sC = (long long)pmat;
            gm.ldC = ld;
            gm.alpha = 1.0;
            gm.beta = 0;
            HIP_TRY(launch_gemm_c64(gm, M));
        }
        int la_cols = kTile, la_K = kTile;   // the look-ahead update of this step: block columns from r0
        double *Lr = Pre, *Li = Pim;           // and its operand: this step's slot, or both slots of the pair
        if (slot == 1) {
            // a'_p: block columns j+1 and j+2 with K = 128, after b_{p-1}, which covers them too
            if (pending_b) HIP_TRY(hipStreamWaitEvent(M, c->la_ev[1 + ((pair - 1) & 1)], 0));
            pending_b = false;
            la_cols = std::min(2 * kTile, ld - r0);
            la_K = 2 * kTile;
            Lr = PPre;
            Li = PPim;
        }
        // the look-ahead's diagonal tile, which the next panel reads (K = 64 at a time on the short-K kernel),
        // after the previous look-ahead's second block column, which covers this tile too
        if (pending_r2) HIP_TRY(hipStreamWaitEvent(M, evR2, 0));
        pending_r2 = false;
        for (int k0 = 0; k0 < la_K; k0 += kTile)
            HIP_TRY(lookahead(Lr + (size_t)k0 * ld, Li + (size_t)k0 * ld, kTile, r0, r0, kTile, kTile, 1, M));
        // b_p on the side stream: every block column from j+3 on, K = 128. It starts after the diagonal tile
        // above, so that the tile the next panel waits for is not queued behind the whole update.
        const int rb = r0 + 2 * kTile;
        if (slot == 1 && rb < ld) {
            HIP_TRY(hipEventRecord(evA, M));
            HIP_TRY(hipStreamWaitEvent(S, evA, 0));
            HerkArgs h{};
            h.Are = PPre;
            h.Aim = PPim;
            h.sA = (long long)pmat;
            h.ldA = ld;
            h.colA = rb;
            h.K = 2 * kTile;
            h.w = nullptr;
            h.sw = 0;
            h.alpha = -1.0;
            h.Cre = cr;
            h.Cim = ci;
            h.sC = ld2;
            h.ldC = ld;
            h.r0 = rb;
            h.nT = (ld - rb) / kTile;
            h.nbatch = nb;
            HIP_TRY(launch_herk_f64(h, S));
            HIP_TRY(hipEventRecord(c->la_ev[1 + (pair & 1)], S));
            pending_b = true;
            last_p = pair;
        }
        // the rest of the look-ahead on S2, beside the next panel
        if (r0 + kTile < ld) {
            HIP_TRY(hipEventRecord(evD, M));
            HIP_TRY(hipStreamWaitEvent(S2, evD, 0));
            // rows below the diagonal tile of the first block column (the next solve waits for these), then
            // (K = 128) the second block column from its own diagonal tile down (the next look-ahead's
            // diagonal tile waits for that); the strict upper part of a diagonal tile is never read
            HIP_TRY(lookahead(Lr, Li, la_K, r0 + kTile, r0, ld - r0 - kTile, kTile, 0, S2));
            HIP_TRY(hipEventRecord(evR, S2));
            pending_r = true;
            if (la_cols > kTile) {
                HIP_TRY(lookahead(Lr, Li, la_K, r0 + kTile, r0 + kTile, ld - r0 - kTile, la_cols - kTile, 0, S2));
                HIP_TRY(hipEventRecord(evR2, S2));
                pending_r2 = true;
            }
        }
    }
    if (pending_r) HIP_TRY(hipStreamWaitEvent(M, evR, 0));
    if (pending_r2) HIP_TRY(hipStreamWaitEvent(M, evR2, 0));
    if (pending_b) HIP_TRY(hipStreamWaitEvent(M, c->la_ev[1 + (last_p & 1)], 0));
    for (int qi = 0; qi < nq; ++qi) {
        QJob& Q = B.qj[q0 + qi];
        HIP_TRY(launch_finalize(logdet + qi * nw, trk + qi * nw, failv + qi * nw,
                                static_cast<const double*>(B.d_ow), nw, Q.F, Q.ec, M));
    }
    return RPA_OK;
}

// E_c of every job of the batch, one class of equal leading dimension after the other
int enqueue_ec_all(Batch& B, bool from_full, const void* chi_full, double* Lblocks = nullptr) {
    for (const QClass& C : B.cls) {
        int rc = enqueue_ec_class(B, C, from_full, chi_full, Lblocks);
        if (rc) return rc;
    }
    return RPA_OK;
}

void remember_fail_flags(Batch& B) {
    char* sm = static_cast<char*>(buf(B, "ec_small"));
    B.c->last_fail = reinterpret_cast<int*>(reinterpret_cast<double*>(sm) + B.qj.size() * 2 * B.nw);
    B.c->last_nw = B.nw;
    B.c->last_nq = (int)B.qj.size();
    B.c->last_qorder.clear();
    for (auto& Q : B.qj) B.c->last_qorder.push_back(Q.orig);
}

int check_common(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs) {
    if (!ctx) return fail(RPA_ERR_INPUT, "NULL context");
    if (nk <= 0 || !k || !kq) return fail(RPA_ERR_INPUT, "need at least one (k, k+q) state-set pair");
    if (!qs) return fail(RPA_ERR_INPUT, "NULL qspec");
    for (int i = 1; i < nk; ++i)
        if (k[i].natoms != k[0].natoms) return fail(RPA_ERR_SHAPE, "atom count differs between k-points");
    return RPA_OK;
}

// plan every (k, q) of a call: validation, tables, one upload, buffer sizes
// qk (optional, nq + 1 entries): q-point j uses the sets qk[j] .. qk[j+1]-1 of k and kq; without it every
// q-point uses all nk of them.
// n-grouped pair tables of the n-factorised MFMA PAW term, one per (k set, chunk size), uploaded beside the
// call's other tables (before any launch or graph capture)
int build_pawn(Batch& B, const char* table_buf) {
    B.pawn.clear();
    if (!B.paw_nform) return RPA_OK;
    Upload up;
    for (auto& Q : B.qj)
        for (size_t ik = 0; ik < B.ks.size(); ++ik) {
            if (!Q.uses((int)ik)) continue;
            const auto key = std::make_pair((int)ik, Q.Pc);
            if (B.pawn.count(key)) continue;
            PawN& T = B.pawn[key];
            const KSet& K = B.ks[ik];
            const int P = (int)K.pn.size();
            T.perm.resize(std::max(P, 1));
            for (int p0 = 0; p0 < P; p0 += Q.Pc) {
                const int np = std::min(Q.Pc, P - p0);
                int nlo = K.pn[p0], nhi = nlo;
                for (int i = p0; i < p0 + np; ++i) {
                    nlo = std::min(nlo, (int)K.pn[i]);
                    nhi = std::max(nhi, (int)K.pn[i]);
                }
                const int nn = nhi - nlo + 1;
                std::vector<int32_t> start(nn + 1, 0);
                for (int i = p0; i < p0 + np; ++i) start[K.pn[i] - nlo + 1]++;
                for (int b = 0; b < nn; ++b) start[b + 1] += start[b];
                std::vector<int32_t> fill(start.begin(), start.end() - 1);
                for (int i = 0; i < np; ++i) T.perm[p0 + fill[K.pn[p0 + i] - nlo]++] = i;
                T.s0.push_back((int32_t)(T.seg.size() / 3));
                T.nlo.push_back(nlo);
                T.nn.push_back(nn);
                for (int b = 0; b < nn; ++b)
                    for (int f = start[b]; f < start[b + 1]; f += 64)
                        T.seg.insert(T.seg.end(), {b, f, std::min(64, start[b + 1] - f)});
                T.ns.push_back((int32_t)(T.seg.size() / 3) - T.s0.back());
            }
            if (T.seg.empty()) T.seg.assign(3, 0);
            up.add(T.perm, &T.d_perm);
            up.add(T.seg, &T.d_seg);
        }
    return do_upload(B.c, up, B.s, (std::string(table_buf) + "_pawn").c_str());
}

int plan_batch(Batch& B, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, int nq,
               bool need_ec, bool need_chi, const char* table_buf, const int32_t* pn = nullptr,
               const int32_t* pm = nullptr, int npairs = -1, const int* qk = nullptr) {
    auto q_uses = [&](int j, int i) { return !qk || (i >= qk[j] && i < qk[j + 1]); };
    rpa_ctx* c = B.c;
    Upload up;
    int rc = prepare_common(B, &k[0], up);
    if (rc) return rc;
    B.ks.resize(nk);
    // sets with a symmetry operation are unfolded once each (a k+q set that is its k set stays shared)
    std::map<const rpa_states*, const rpa_states*> unfolded;
    auto resolve = [&](const rpa_states* s, const std::string& tag, const rpa_states** out) -> int {
        if (!s->sym) {
            *out = s;
            return RPA_OK;
        }
        auto it = unfolded.find(s);
        if (it != unfolded.end()) {
            *out = it->second;
            return RPA_OK;
        }
        int r = check_states(c, s, tag.c_str());
        if (r) return r;
        r = unfold_set(B, s, tag, up, out);
        if (r) return r;
        unfolded[s] = *out;
        return RPA_OK;
    };
    for (int i = 0; i < nk; ++i) {
        rc = resolve(&k[i], "k" + std::to_string(i), &B.ks[i].k);
        if (rc) return rc;
        if (same_set(&k[i], &kq[i]) && k[i].sym == kq[i].sym) {
            B.ks[i].kq = B.ks[i].k;
        } else {
            rc = resolve(&kq[i], "kq" + std::to_string(i), &B.ks[i].kq);
            if (rc) return rc;
        }
        for (int j = 0; j < nq; ++j) {
            if (!q_uses(j, i)) continue;
            rc = check_pair(c, B.ks[i].k, B.ks[i].kq, &qs[j]);
            if (rc) return rc;
        }
        rc = prepare_kset(B, B.ks[i], up, pn, pm, npairs);
        if (rc) return rc;
        // the optical head divides by eps_m - eps_n (Eq. n_q0): no degenerate transition
        bool optical = false;
        for (int j = 0; j < nq; ++j) optical = optical || (qs[j].optical && q_uses(j, i));
        const KSet& K = B.ks[i];
        for (size_t p = 0; optical && p < K.pn.size(); ++p)
            if (K.k->eps[K.pn[p]] == K.kq->eps[K.pm[p]])
                return fail(RPA_ERR_INPUT, "optical limit with a degenerate transition (n = " + std::to_string(K.pn[p]) +
                                               ", m = " + std::to_string(K.pm[p]) + ": eps_m == eps_n)");
    }
    // every q-point's plan, then the jobs in class order (leading dimension descending, caller's order
    // within a class); the uploads point into the jobs, so they are registered after the reordering
    // q-points that share every (k, k+q) set share the product conj(phi_n) phi_m of each pair and its
    // transform along x and y (Eq. fft: only the sphere differs from q to q), so the kept (m1, m2) box is the
    // union of the spheres' boxes and the transform runs once per chunk for all of them
    int ubox[4] = {0, 0, 0, 0};
    B.share_xy = false;
    if (!qk && nq > 1 && B.allow_share_xy) {
        bool ok = true;
        for (int j = 0; j < nq && ok; ++j) {
            if (qs[j].NG <= 0 || !qs[j].gmiller) {
                ok = false;
                break;
            }
            int lo[3], hi[3];
            sphere_box(&qs[j], lo, hi);
            if (j == 0) {
                ubox[0] = lo[0]; ubox[1] = hi[0]; ubox[2] = lo[1]; ubox[3] = hi[1];
            } else {
                ubox[0] = std::min(ubox[0], lo[0]); ubox[1] = std::max(ubox[1], hi[0]);
                ubox[2] = std::min(ubox[2], lo[1]); ubox[3] = std::max(ubox[3], hi[1]);
            }
        }
        B.share_xy = ok && ubox[1] - ubox[0] + 1 <= c->N[0] && ubox[3] - ubox[2] + 1 <= c->N[1];
    }
    std::vector<QPlan> plans(nq);
    std::vector<int> order(nq);
    for (int j = 0; j < nq; ++j) {
        rc = plan_q(c, &qs[j], plans[j], need_ec, B.share_xy ? ubox : nullptr);
        if (rc) return rc;
        order[j] = j;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return class_ld(plans[a].NGp, nq) > class_ld(plans[b].NGp, nq);
    });
    B.qj.resize(nq);
    B.cls.clear();
    for (int i = 0; i < nq; ++i) {
        const int j = order[i];
        QJob& Q = B.qj[i];
        Q.qs = &qs[j];
        Q.orig = j;
        if (qk) {
            Q.k0 = qk[j];
            Q.k1 = qk[j + 1];
        }
        Q.qp = std::move(plans[j]);
        Q.ld = class_ld(Q.qp.NGp, nq);
        if (B.cls.empty() || B.cls.back().ld != Q.ld) B.cls.push_back(QClass{Q.ld, i, 0, nullptr, nullptr});
        B.cls.back().nq += 1;
        rc = prepare_q(B, Q, up);
        if (rc) return rc;
    }
    rc = do_upload(c, up, B.s, table_buf);
    if (rc) return rc;
    WorkSizes W;
    rc = presize(B, need_ec, need_chi, W);
    if (rc) return rc;
    return build_pawn(B, table_buf);
}

// ------------------------------------------------------------ the adjoint
struct Csr {
    std::vector<int32_t> start, list;
};

// pairs [p0, p0+np) grouped by band (key = pn or pm) over the window [lo, hi]
Csr group_pairs(const std::vector<int32_t>& key, int p0, int np, int lo, int hi, bool local) {
    Csr c;
    c.start.assign(hi - lo + 2, 0);
    for (int i = 0; i < np; ++i) c.start[key[p0 + i] - lo + 1]++;
    for (int b = 0; b <= hi - lo; ++b) c.start[b + 1] += c.start[b];
    c.list.resize(np);
    std::vector<int32_t> fill(c.start.begin(), c.start.end() - 1);
    for (int i = 0; i < np; ++i) c.list[fill[key[p0 + i] - lo]++] = local ? i : p0 + i;
    return c;
}

// The owner groups of a chunk cut into segments of at most sg pairs for the register x-y adjoint: one
// workgroup per segment and z-plane. An owner with several segments sends each to a partial slot, which the
// reduce kernel adds in afterwards (in slot order, so the result does not depend on the schedule).
struct SegTab {
    std::vector<int32_t> seg;          // per segment: owner, first, end (into the group's list), slot or -1
    std::vector<int32_t> own, ostart;  // owners with several segments, and the ranges of their slots
    int nseg = 0, nslots = 0;
    void *d_seg = nullptr, *d_own = nullptr, *d_ostart = nullptr;
};

int count_slots(const Csr& c, int sg) {
    int n = 0;
    for (size_t b = 0; b + 1 < c.start.size(); ++b) {
        const int cnt = c.start[b + 1] - c.start[b];
        if (cnt > sg) n += (cnt + sg - 1) / sg;
    }
    return n;
}

// segments of at most 16 pairs, longer where the partial slots would pass slot_cap
SegTab make_segments(const Csr& c, int slot_cap) {
    int sg = 16;
    while (count_slots(c, sg) > slot_cap) sg *= 2;
    SegTab t;
    t.ostart.push_back(0);
    for (size_t b = 0; b + 1 < c.start.size(); ++b) {
        const int e0 = c.start[b], e1 = c.start[b + 1], cnt = e1 - e0;
        if (cnt <= 0) continue;
        const bool split = cnt > sg;
        for (int e = e0; e < e1; e += sg) {
            t.seg.insert(t.seg.end(), {(int32_t)b, e, std::min(e + sg, e1), split ? t.nslots++ : -1});
            t.nseg++;
        }
        if (split) {
            t.own.push_back((int32_t)b);
            t.ostart.push_back(t.nslots);
        }
    }
    return t;
}

struct BwChunk {
    int p0, np, nlo, nhi, mlo, mhi;
    Csr byn, bym;
    SegTab sn, sm;
    void *d_ns = nullptr, *d_nl = nullptr, *d_ms = nullptr, *d_ml = nullptr;
};

// gradient outputs of one state set (offsets into the caller's concatenated arrays)
struct BwOut {
    double* deps = nullptr;
    double* dC = nullptr;
    double* dP = nullptr;
};

// host tables of one (k, k+q) set pair: per-chunk band groupings and the global ones for the energies
struct BwSet {
    std::vector<BwChunk> ch;
    Csr gn, gm;
    void *d_gns = nullptr, *d_gnl = nullptr, *d_gms = nullptr, *d_gml = nullptr;
};

// The forward pass (chi0 of every set, E_c, the Cholesky factor, W(w)) once, then every set's pairs are
// recomputed chunk by chunk and taken back to its eps, C and P. outk[i] / outkq[i]: the gradient slots of
// the k and k+q set of pair i (for a k+q set that is its k set, both roles go to outk[i]).
int backward(Batch& B, const double* dEc, double* ec_dev, const std::vector<BwOut>& outk,
             const std::vector<BwOut>& outkq) {
    rpa_ctx* c = B.c;
    QJob& Q = B.qj[0];
    const PairGeom& g = Q.qp.g;
    const int NG = Q.qp.NG, NGp = Q.qp.NGp, nw = B.nw;
    const int nproj = nproj_total(B.ks[0].k);
    const size_t vol = (size_t)c->N[0] * c->N[1] * c->N[2];
    const int Pc = Q.Pc;
    const size_t nks = B.ks.size();
    std::vector<BwSet> sets(nks);
    int maxm = 1, maxn = 1, maxP = 1;
    size_t maxphib = 1;
    // register x-y adjoint: partial slots of one orbital volume each, at most about 2 GiB of them
    const bool reg_adj = c->pair_reg && xyadj_reg_supported(g);
    const int slot_cap = (int)std::max<size_t>(1, ((size_t)2 << 30) / (vol * sizeof(cplx<double>)));
    int maxslots = 1;
    for (size_t ik = 0; ik < nks; ++ik) {
        KSet& K = B.ks[ik];
        BwSet& S = sets[ik];
        const int P = (int)K.pn.size();
        const bool same = same_set(K.k, K.kq);
        const int nbk = K.k->nbands, nbq = K.kq->nbands;
        for (int p0 = 0; p0 < P; p0 += Pc) {
            BwChunk x;
            x.p0 = p0;
            x.np = std::min(Pc, P - p0);
            x.nlo = x.nhi = K.pn[p0];
            x.mlo = x.mhi = K.pm[p0];
            for (int i = p0; i < p0 + x.np; ++i) {
                x.nlo = std::min(x.nlo, (int)K.pn[i]);
                x.nhi = std::max(x.nhi, (int)K.pn[i]);
                x.mlo = std::min(x.mlo, (int)K.pm[i]);
                x.mhi = std::max(x.mhi, (int)K.pm[i]);
            }
            x.byn = group_pairs(K.pn, p0, x.np, x.nlo, x.nhi, true);
            x.bym = group_pairs(K.pm, p0, x.np, x.mlo, x.mhi, true);
            if (reg_adj) {
                x.sn = make_segments(x.byn, slot_cap);
                x.sm = make_segments(x.bym, slot_cap);
                maxslots = std::max({maxslots, x.sn.nslots, x.sm.nslots});
            }
            maxm = std::max(maxm, x.mhi - x.mlo + 1);
            maxn = std::max(maxn, x.nhi - x.nlo + 1);
            S.ch.push_back(std::move(x));
        }
        S.gn = group_pairs(K.pn, 0, P, 0, nbk - 1, false);
        S.gm = group_pairs(K.pm, 0, P, 0, nbq - 1, false);
        maxP = std::max(maxP, P);
        maxphib = std::max(maxphib, (size_t)(nbk + (same ? 0 : nbq)) * vol);
    }

    // buffers (sized for every set); the products W(w) rho of all frequencies in one batched GEMM per run
    // of at most kYRows pairs of a chunk (and at most 8 GiB of products)
    constexpr int kYRows = 4096;
    const size_t yrow = 2 * (size_t)NGp * 8 * nw;   // bytes of one pair's products, all frequencies
    const int yrows = (int)std::max<size_t>(1, std::min<size_t>({(size_t)Pc, (size_t)kYRows, ((size_t)8 << 30) / yrow}));
    const size_t ybytes = 2 * (size_t)yrows * NGp * 8;   // one frequency's products of a run
    const size_t mat = (size_t)nw * NGp * NGp;
    void *pB, *pX, *pL, *pY, *pG, *pdE, *pu, *pcw, *pZ, *pU, *pgn, *pT, *pPb, *pPart;
    struct NB {
        const char* n;
        size_t b;
        void** p;
    } list[] = {{"bw_B", 2 * mat * 8, &pB}, {"bw_X", 2 * mat * 8, &pX},
                {"bw_L", (size_t)(NGp / kTile) * 2 * nw * kTile * kTile * 8, &pL},
                {"bw_Y", ybytes * nw, &pY}, {"bw_g", 2 * (size_t)Pc * NGp * 8, &pG},
                {"bw_dEda", (size_t)nw * ((Pc + 3) / 4 * 4) * 8, &pdE}, {"bw_u", (size_t)maxP * 8, &pu},
                {"bw_cw", 64 * 8, &pcw}, {"bw_Z", 4 * (size_t)Pc * std::max(nproj, 1) * 8, &pZ},
                {"bw_U", 2 * (size_t)maxm * std::max(nproj, 1) * NGp * 8, &pU}, {"bw_gnum", 2 * (size_t)Pc * 8, &pgn},
                {"bw_tadj", (size_t)Pc * g.N3 * g.ncols * 16, &pT}, {"bw_phibar", maxphib * 16, &pPb},
                {"bw_part", reg_adj ? (size_t)maxslots * vol * 16 : 16, &pPart}};
    for (auto& e : list) {
        int rc = get_buf(c, e.n, e.b, B.s, e.p);
        if (rc) return rc;
    }
    double* Lb = static_cast<double*>(pL);
    double *Br_ = static_cast<double*>(pB), *Bi_ = Br_ + mat;
    double *Xr = static_cast<double*>(pX), *Xi = Xr + mat;
    double *Yr = static_cast<double*>(pY), *Yi = Yr + (size_t)yrows * NGp;
    double *gr = static_cast<double*>(pG), *gi = gr + (size_t)Pc * NGp;
    double* dEda = static_cast<double*>(pdE);
    double* u = static_cast<double*>(pu);
    double* cw = static_cast<double*>(pcw);
    double *Zm = static_cast<double*>(pZ), *Zn = Zm + 2 * (size_t)Pc * std::max(nproj, 1);
    double *Ur = static_cast<double*>(pU), *Ui = Ur + (size_t)maxm * std::max(nproj, 1) * NGp;
    double* gnum = static_cast<double*>(pgn);
    cplx<double>* tadj = static_cast<cplx<double>*>(pT);
    cplx<double>* part = static_cast<cplx<double>*>(pPart);
    (void)maxn;

    // forward: chi0, E_c, and the factor L with its inverted diagonal blocks
    int rc = enqueue_chi0<double>(B);
    if (rc) return rc;
    Q.ec = ec_dev;
    Q.F = nullptr;
    rc = enqueue_ec_all(B, false, nullptr, Lb);
    if (rc) return rc;
    remember_fail_flags(B);
    {
    ProfScope ps_(c, S_BW_INV, B.s);
    // X = L^-1 by blocked substitution on the identity, then (1 - K)^-1 = X^H X
    HIP_TRY(launch_identity(Br_, Bi_, NGp, NGp, nw, B.s));
    HIP_TRY(launch_zero_d(Xr, 2 * mat, B.s));  // columns right of each block row stay zero
    const int nblk = NGp / kTile;
    for (int i = 0; i < nblk; ++i) {
        const int ncol = (i + 1) * kTile;
        GemmArgs g1{};
        g1.M = kTile; g1.N = ncol; g1.K = kTile; g1.nbatch = nw;
        g1.Ar = Lb + (size_t)i * 2 * nw * kTile * kTile; g1.Ai = g1.Ar + (size_t)nw * kTile * kTile;
        g1.sA = kTile * kTile; g1.aI = kTile; g1.aK = 1;
        g1.Br = Br_ + (size_t)i * kTile * NGp; g1.Bi = Bi_ + (size_t)i * kTile * NGp;
        g1.sB = (long long)NGp * NGp; g1.bK = NGp; g1.bJ = 1;
        g1.Cr = Xr + (size_t)i * kTile * NGp; g1.Ci = Xi + (size_t)i * kTile * NGp;
        g1.sC = (long long)NGp * NGp; g1.ldC = NGp; g1.alpha = 1.0; g1.beta = 0;
        HIP_TRY(launch_gemm_c64(g1, B.s));
        const int r1 = (i + 1) * kTile;
        if (r1 < NGp) {
            GemmArgs g2{};
            g2.M = NGp - r1; g2.N = ncol; g2.K = kTile; g2.nbatch = nw;
            g2.Ar = Q.cr + (size_t)r1 * NGp + i * kTile; g2.Ai = Q.ci + (size_t)r1 * NGp + i * kTile;
            g2.sA = (long long)NGp * NGp; g2.aI = NGp; g2.aK = 1;
            g2.Br = g1.Cr; g2.Bi = g1.Ci; g2.sB = (long long)NGp * NGp; g2.bK = NGp; g2.bJ = 1;
            g2.Cr = Br_ + (size_t)r1 * NGp; g2.Ci = Bi_ + (size_t)r1 * NGp;
            g2.sC = (long long)NGp * NGp; g2.ldC = NGp; g2.alpha = -1.0; g2.beta = 1;
            HIP_TRY(launch_gemm_c64(g2, B.s));
        }
    }
    {
        GemmArgs g3{};
        g3.M = NGp; g3.N = NGp; g3.K = NGp; g3.nbatch = nw;
        g3.Ar = Xr; g3.Ai = Xi; g3.sA = (long long)NGp * NGp; g3.aI = 1; g3.aK = NGp; g3.conjA = 1;
        g3.Br = Xr; g3.Bi = Xi; g3.sB = (long long)NGp * NGp; g3.bK = NGp; g3.bJ = 1;
        g3.Cr = Br_; g3.Ci = Bi_; g3.sC = (long long)NGp * NGp; g3.ldC = NGp; g3.alpha = 1.0; g3.beta = 0;
        // X is lower triangular: the lower half of X^H X, with k from the tile's first row (W is built from
        // that half and mirrored)
        g3.lower = 1;
        g3.ktri = 1;
        HIP_TRY(launch_gemm_c64(g3, B.s));
    }
    HIP_TRY(launch_build_w(Br_, Bi_, NG, NGp, nw, static_cast<const double*>(Q.d_vs), B.s));
    HIP_TRY(launch_freq_coeffs(dEc, static_cast<const double*>(B.d_ow), nw, cw, B.s));
    }

    const int lda = (Pc + 3) / 4 * 4;
    double* rre = static_cast<double*>(buf(B, "rho"));
    double* rim = rre + (size_t)Pc * NGp;
    double* aw = static_cast<double*>(buf(B, "weights"));
    for (size_t ik = 0; ik < nks; ++ik) {
        KSet& K = B.ks[ik];
        BwSet& S = sets[ik];
        const int P = (int)K.pn.size();
        const bool same = same_set(K.k, K.kq);
        const int nbk = K.k->nbands, nbq = K.kq->nbands;
        double* deps_k = outk[ik].deps;
        double* dC_k = outk[ik].dC;
        double* dP_k = outk[ik].dP;
        double* deps_kq = same ? deps_k : outkq[ik].deps;
        double* dC_kq = same ? dC_k : outkq[ik].dC;
        double* dP_kq = same ? dP_k : outkq[ik].dP;
        // this set's outputs start at zero (a set with no transitions keeps a zero gradient)
        std::optional<ProfScope> pz_(std::in_place, c, S_BW_REST, B.s);
        HIP_TRY(launch_zero_d(deps_k, nbk, B.s));
        HIP_TRY(launch_zero_d(dC_k, 2 * (size_t)nbk * K.k->nQ, B.s));
        if (nproj) HIP_TRY(launch_zero_d(dP_k, 2 * (size_t)nbk * nproj, B.s));
        if (!same) {
            HIP_TRY(launch_zero_d(deps_kq, nbq, B.s));
            HIP_TRY(launch_zero_d(dC_kq, 2 * (size_t)nbq * K.kq->nQ, B.s));
            if (nproj) HIP_TRY(launch_zero_d(dP_kq, 2 * (size_t)nbq * nproj, B.s));
        }
        if (P == 0) continue;
        Upload up;
        for (auto& x : S.ch) {
            up.add(x.byn.start, &x.d_ns);
            up.add(x.byn.list, &x.d_nl);
            up.add(x.bym.start, &x.d_ms);
            up.add(x.bym.list, &x.d_ml);
            if (reg_adj) {
                for (SegTab* t : {&x.sn, &x.sm}) {
                    up.add(t->seg, &t->d_seg);
                    if (!t->own.empty()) {
                        up.add(t->own, &t->d_own);
                        up.add(t->ostart, &t->d_ostart);
                    }
                }
            }
        }
        up.add(S.gn.start, &S.d_gns);
        up.add(S.gn.list, &S.d_gnl);
        up.add(S.gm.start, &S.d_gms);
        up.add(S.gm.list, &S.d_gml);
        rc = do_upload(c, up, B.s, "bw_tables");
        if (rc) return rc;
        cplx<double>* phib_k = static_cast<cplx<double>*>(pPb);
        cplx<double>* phib_kq = same ? phib_k : phib_k + (size_t)nbk * vol;
        HIP_TRY(launch_zero_d(reinterpret_cast<double*>(phib_k), 2 * (size_t)(nbk + (same ? 0 : nbq)) * vol, B.s));
        HIP_TRY(launch_zero_d(u, std::max(P, 1), B.s));
        pz_.reset();
        // this set's orbitals (the forward pass left those of the last set in the buffers)
        cplx<double>* phik_c = nullptr;
        cplx<double>* phikq_c = nullptr;
        if (nks > 1) {
            rc = enqueue_orbitals<double>(B, K.k, K.d_mapk, K.zcolk, K.d_zcolk, "phi_k", &phik_c);
            if (rc) return rc;
            if (!same) {
                rc = enqueue_orbitals<double>(B, K.kq, K.d_mapkq, K.zcolkq, K.d_zcolkq, "phi_kq", &phikq_c);
                if (rc) return rc;
            }
        }
        const double* phik = static_cast<const double*>(buf(B, "phi_k"));
        const double* phikq = same ? phik : static_cast<const double*>(buf(B, "phi_kq"));
        const double prefac = K.k->weight / c->volume;
        for (auto& x : S.ch) {
            const int p0 = x.p0, np = x.np;
            const int32_t* pn = static_cast<const int32_t*>(K.d_pn) + p0;
            const int32_t* pm = static_cast<const int32_t*>(K.d_pm) + p0;
            rc = enqueue_pairs<double>(B, Q, K, (int)ik, reinterpret_cast<const cplx<double>*>(phik),
                                       reinterpret_cast<const cplx<double>*>(phikq), p0, np, rre, rim);
            if (rc) return rc;
            std::optional<ProfScope> pr_(std::in_place, c, S_BW_REST, B.s);
            HIP_TRY(launch_weights(static_cast<const double*>(K.d_epsk), static_cast<const double*>(K.d_epskq),
                                   static_cast<const double*>(K.d_fk), static_cast<const double*>(K.d_fkq), pn, pm,
                                   np, static_cast<const double*>(B.d_om), nw, prefac, aw, lda, B.s));
            HIP_TRY(launch_zero_d(gr, 2 * (size_t)Pc * NGp, B.s));
            pr_.reset();
            for (int r0 = 0; r0 < np; r0 += yrows) {
                const int nr = std::min(yrows, np - r0);
                GemmArgs gy{};
                gy.M = nr; gy.N = NGp; gy.K = NGp; gy.nbatch = nw;
                gy.Ar = rre + (size_t)r0 * NGp; gy.Ai = rim + (size_t)r0 * NGp; gy.sA = 0; gy.aI = NGp; gy.aK = 1;
                gy.Br = Br_; gy.Bi = Bi_; gy.sB = (long long)NGp * NGp; gy.bK = 1; gy.bJ = NGp;
                gy.Cr = Yr; gy.Ci = Yi; gy.sC = (long long)(ybytes / 8); gy.ldC = NGp; gy.alpha = 1.0; gy.beta = 0;
                {
                    ProfScope pg_(c, S_BW_GEMM, B.s);
                    HIP_TRY(launch_gemm_c64(gy, B.s));
                }
                ProfScope pw_(c, S_BW_REST, B.s);
                HIP_TRY(launch_grad_weights_all(rre + (size_t)r0 * NGp, rim + (size_t)r0 * NGp, Yr, Yi, ybytes / 8, NG,
                                                NGp, aw + r0, lda, nw, cw, gr + (size_t)r0 * NGp,
                                                gi + (size_t)r0 * NGp, dEda + r0, nr, B.s));
            }
            pr_.emplace(c, S_BW_REST, B.s);
            HIP_TRY(launch_pair_eps(dEda, lda, nw, static_cast<const double*>(K.d_epsk),
                                    static_cast<const double*>(K.d_epskq), static_cast<const double*>(K.d_fk),
                                    static_cast<const double*>(K.d_fkq), pn, pm, np,
                                    static_cast<const double*>(B.d_om), prefac, u + p0, B.s));
            const bool opt = Q.qs->optical && Q.qp.g0 >= 0;
            if (opt)
                HIP_TRY(launch_optical_adj(rre, rim, gr, gi, Q.qp.g0, NGp, static_cast<const double*>(K.d_epsk),
                                           static_cast<const double*>(K.d_epskq), pn, pm, np, u + p0, gnum, B.s));
            const int32_t* ns = static_cast<const int32_t*>(x.d_ns);
            const int32_t* nl = static_cast<const int32_t*>(x.d_nl);
            const int32_t* ms = static_cast<const int32_t*>(x.d_ms);
            const int32_t* ml = static_cast<const int32_t*>(x.d_ml);
            const int nn = x.nhi - x.nlo + 1, nm = x.mhi - x.mlo + 1;
            if (nproj > 0) {
                double* Yn = static_cast<double*>(buf(B, "paw_y"));
                double* Yni = Yn + (size_t)nn * nproj * NGp;
                HIP_TRY(launch_paw_y<double>(static_cast<const double*>(K.k->P), nproj,
                                             static_cast<const int32_t*>(K.d_nlist) + x.nlo, nn,
                                             static_cast<const int32_t*>(B.d_poff),
                                             static_cast<const int32_t*>(B.d_qoff), K.k->natoms, nproj,
                                             static_cast<const double*>(Q.qs->Qpaw), NG, NGp, Yn, Yni, B.s));
                HIP_TRY(launch_paw_u(static_cast<const double*>(K.kq->P), nproj, x.mlo, nm,
                                     static_cast<const int32_t*>(B.d_poff), static_cast<const int32_t*>(B.d_qoff),
                                     K.k->natoms, nproj, static_cast<const double*>(Q.qs->Qpaw), NG, NGp, Ur, Ui,
                                     B.s));
                HIP_TRY(launch_paw_adj(gr, gi, NG, NGp, Yn, Yni, x.nlo, Ur, Ui, x.mlo, nproj, pn, pm, np, Zm, Zn,
                                       B.s));
                HIP_TRY(launch_paw_reduce(Zn, ns, nl, nn, nproj, dP_k, x.nlo, opt ? gnum : nullptr,
                                          static_cast<const double*>(K.kq->P), pm, static_cast<const double*>(Q.d_Dq),
                                          static_cast<const int32_t*>(B.d_poff),
                                          static_cast<const int32_t*>(B.d_qoff), K.k->natoms, 0, B.s));
                HIP_TRY(launch_paw_reduce(Zm, ms, ml, nm, nproj, dP_kq, x.mlo, opt ? gnum : nullptr,
                                          static_cast<const double*>(K.k->P), pn, static_cast<const double*>(Q.d_Dq),
                                          static_cast<const int32_t*>(B.d_poff),
                                          static_cast<const int32_t*>(B.d_qoff), K.k->natoms, 1, B.s));
            }
            if (opt) {
                const double* wq = static_cast<const double*>(Q.d_wq[ik]);
                HIP_TRY(launch_optical_c(gnum, ns, nl, pm, static_cast<const double*>(K.kq->C), K.k->nQ, wq, 0, nn,
                                         dC_k + 2 * (size_t)x.nlo * K.k->nQ, B.s));
                HIP_TRY(launch_optical_c(gnum, ms, ml, pn, static_cast<const double*>(K.k->C), K.kq->nQ, wq, 1, nm,
                                         dC_kq + 2 * (size_t)x.mlo * K.kq->nQ, B.s));
            }
            pr_.reset();
            ProfScope pa_(c, S_BW_PAIRS, B.s);
            HIP_TRY(launch_zadj(gr, gi, NGp, np, g, static_cast<const int32_t*>(Q.d_cs),
                                static_cast<const int32_t*>(Q.d_cg), static_cast<const int32_t*>(Q.d_ckz),
                                static_cast<const cplx<double>*>(B.d_tw[2]), tadj, B.s));
            if (reg_adj) {
                auto side = [&](const SegTab& t, const int32_t* lst, const int32_t* oth, const double* phio, int band0,
                                int sd, cplx<double>* phib) -> hipError_t {
                    hipError_t e = launch_xyadj_reg(tadj, g, static_cast<const int32_t*>(t.d_seg), t.nseg, lst, oth,
                                                    reinterpret_cast<const cplx<double>*>(phio), band0, sd, phib,
                                                    part, B.s);
                    if (e != hipSuccess) return e;
                    return launch_xyadj_reduce(part, vol, static_cast<const int32_t*>(t.d_own),
                                               static_cast<const int32_t*>(t.d_ostart), (int)t.own.size(), band0,
                                               phib, B.s);
                };
                HIP_TRY(side(x.sm, ml, pn, phik, x.mlo, 1, phib_kq));
                HIP_TRY(side(x.sn, nl, pm, phikq, x.nlo, 0, phib_k));
            } else {
                HIP_TRY(launch_xyadj(tadj, g, ms, ml, pn, reinterpret_cast<const cplx<double>*>(phik), x.mlo, nm, 1,
                                     static_cast<const int32_t*>(Q.d_kx), static_cast<const int32_t*>(Q.d_ky),
                                     static_cast<const cplx<double>*>(B.d_tw[0]),
                                     static_cast<const cplx<double>*>(B.d_tw[1]), phib_kq, B.s));
                HIP_TRY(launch_xyadj(tadj, g, ns, nl, pm, reinterpret_cast<const cplx<double>*>(phikq), x.nlo, nn, 0,
                                     static_cast<const int32_t*>(Q.d_kx), static_cast<const int32_t*>(Q.d_ky),
                                     static_cast<const cplx<double>*>(B.d_tw[0]),
                                     static_cast<const cplx<double>*>(B.d_tw[1]), phib_k, B.s));
            }
        }
        // energies
        ProfScope pe_(c, S_BW_REST, B.s);
        HIP_TRY(launch_eps_reduce(u, static_cast<const int32_t*>(S.d_gns), static_cast<const int32_t*>(S.d_gnl), nbk,
                                  1.0, deps_k, B.s));
        HIP_TRY(launch_eps_reduce(u, static_cast<const int32_t*>(S.d_gms), static_cast<const int32_t*>(S.d_gml), nbq,
                                  -1.0, deps_kq, B.s));
        // coefficients: C_bar = unnormalised forward DFT of phi_bar, read at the plane-wave Miller indices:
        // x and y on every plane, then z on the columns that hold coefficients (register-resident lines
        // where the axis length has them, LDS passes otherwise)
        for (int side = 0; side < (same ? 1 : 2); ++side) {
            cplx<double>* ph = side == 0 ? phib_k : phib_kq;
            const int nb = side == 0 ? nbk : nbq;
            const std::vector<int32_t>& zc = side == 0 ? K.zcolk : K.zcolkq;
            const int32_t* d_zc = static_cast<const int32_t*>(side == 0 ? K.d_zcolk : K.d_zcolkq);
            hipError_t e = c->pair_reg ? launch_grid_fft_xy_reg<double>(ph, nb, c->N[0], c->N[1], c->N[2], -1, B.s)
                                       : hipErrorNotSupported;
            if (e == hipErrorNotSupported) {
                for (int ax = 0; ax < 2; ++ax)
                    HIP_TRY(launch_fft_axis<double>(ph, nb, c->N[0], c->N[1], c->N[2], ax, c->plan[ax],
                                                    static_cast<const cplx<double>*>(B.d_tw[ax]), -1, B.s));
            } else {
                HIP_TRY(e);
            }
            e = c->pair_reg ? launch_grid_fft_z_reg<double>(ph, nb, c->N[0], c->N[1], c->N[2], -1, d_zc,
                                                            (int)zc.size(), B.s)
                            : hipErrorNotSupported;
            if (e == hipErrorNotSupported)
                HIP_TRY(launch_fft_axis<double>(ph, nb, c->N[0], c->N[1], c->N[2], 2, c->plan[2],
                                                static_cast<const cplx<double>*>(B.d_tw[2]), -1, B.s));
            else
                HIP_TRY(e);
        }
        HIP_TRY(launch_gather_c(phib_k, vol, static_cast<const int32_t*>(K.d_mapk), K.k->nQ, nbk, dC_k, B.s));
        // with one state set both roles accumulated into the same phi_bar above
        if (!same)
            HIP_TRY(launch_gather_c(phib_kq, vol, static_cast<const int32_t*>(K.d_mapkq), K.kq->nQ, nbq, dC_kq,
                                    B.s));
    }
    return RPA_OK;
}

// key of a batched call: every host value the captured launches baked in, and
// every device pointer they read or write
uint64_t batch_key(const rpa_states* k, const rpa_states* kq, int nk, int nq, const rpa_qspec* qs, const rpa_freq* fr,
                   rpa_precision prec, const double* ec, const double* F, void* stream) {
    Fnv h;
    h.val(nk);
    h.val(nq);
    h.val(prec);
    h.val(ec);
    h.val(F);
    h.val(stream);
    auto st = [&](const rpa_states* s) {
        h.val(s->nbands);
        h.val(s->nQ);
        h.val(s->C);
        h.val(s->P);
        h.val(s->natoms);
        h.bytes(s->miller, sizeof(int32_t) * 3 * (size_t)s->nQ);
        h.bytes(s->eps, sizeof(double) * s->nbands);
        h.bytes(s->f, sizeof(double) * s->nbands);
        if (s->natoms > 0) h.bytes(s->proj_off, sizeof(int32_t) * (s->natoms + 1));
        h.bytes(s->kpt, sizeof(s->kpt));
        h.val(s->weight);
        h.val(s->dfde != nullptr);
        if (s->dfde) h.bytes(s->dfde, sizeof(double) * s->nbands);
        h.val(s->sym != nullptr);
        if (s->sym) {
            const rpa_symop* o = s->sym;
            h.bytes(o->rot, sizeof(o->rot));
            h.val(o->time_reversal);
            h.bytes(o->gshift, sizeof(o->gshift));
            h.bytes(o->kibz, sizeof(o->kibz));
            if (s->natoms > 0 && o->atom_map && o->atom_shift && o->proj_rot) {
                h.bytes(o->atom_map, sizeof(int32_t) * s->natoms);
                h.bytes(o->atom_shift, sizeof(int32_t) * 3 * s->natoms);
                size_t nd = 0;
                for (int a = 0; a < s->natoms; ++a) {
                    const size_t np = (size_t)(s->proj_off[a + 1] - s->proj_off[a]);
                    nd += np * np;
                }
                h.bytes(o->proj_rot, sizeof(double) * nd);
            }
        }
    };
    for (int i = 0; i < nk; ++i) {
        st(&k[i]);
        st(&kq[i]);
    }
    for (int j = 0; j < nq; ++j) {
        const rpa_qspec& q = qs[j];
        h.bytes(q.q, sizeof(q.q));
        h.val(q.optical);
        h.bytes(q.qhat, sizeof(q.qhat));
        h.val(q.NG);
        h.bytes(q.gmiller, sizeof(int32_t) * 3 * (size_t)q.NG);
        h.val(q.Qpaw);
        h.val(q.weight);
        if (q.optical && q.Dpaw && k[0].natoms > 0) {
            int nq2 = 0;
            for (int a = 0; a < k[0].natoms; ++a) {
                const int np = k[0].proj_off[a + 1] - k[0].proj_off[a];
                nq2 += np * np;
            }
            h.bytes(q.Dpaw, sizeof(double) * 3 * (size_t)nq2);
        }
    }
    h.val(fr->nw);
    h.bytes(fr->omega, sizeof(double) * fr->nw);
    h.bytes(fr->weight, sizeof(double) * fr->nw);
    return h.h;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char* rpa_status_string(int status) {
    switch (status) {
        case RPA_OK: return "ok";
        case RPA_ERR_INPUT: return "invalid input";
        case RPA_ERR_SHAPE: return "inconsistent shapes";
        case RPA_ERR_ALIAS: return "grid too small for an alias-free pair product";
        case RPA_ERR_NOMEM: return "out of device memory or workspace cap";
        case RPA_ERR_NOT_PD: return "1 - K not positive definite";
        case RPA_ERR_HIP: return "HIP runtime error";
        case RPA_ERR_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* rpa_last_error(const rpa_ctx*) { return g_err.c_str(); }

int rpa_create(rpa_ctx** out, const rpa_cell* cell, int device, size_t cap) {
    if (!out || !cell) return fail(RPA_ERR_INPUT, "NULL argument");
    *out = nullptr;
    FftPlan plans[3];
    int rc = check_grid(cell, plans);
    if (rc) return rc;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(RPA_ERR_INPUT, "no such device");
    HIP_TRY(hipSetDevice(device));
    rpa_ctx* c = new rpa_ctx();
    c->device = device;
    std::memcpy(c->A, cell->A, sizeof(c->A));
    for (int i = 0; i < 3; ++i) {
        c->N[i] = cell->n[i];
        c->plan[i] = plans[i];
    }
    reciprocal(c->A, c->B);
    c->volume = std::fabs(det3(c->A));
    c->cap = cap;
    if (hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return fail(RPA_ERR_HIP, "hipEventCreate failed");
    }
    // set-up for the allocation-free entry point: this device's scratch address and the Cholesky
    // look-ahead streams, so that no call has to create them later
    rc = scratch_address(device, &c->scratch);
    if (!rc) rc = ensure_lookahead(c);
    if (rc) {
        const std::string msg = g_err;
        rpa_destroy(c);
        return fail(rc, msg);
    }
    *out = c;
    return RPA_OK;
}

int rpa_destroy(rpa_ctx* c) {
    if (!c) return RPA_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->la_stream) (void)hipStreamDestroy(c->la_stream);
    if (c->la2_stream) (void)hipStreamDestroy(c->la2_stream);
    for (hipEvent_t e : c->la2_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->la_ev)
        if (e) (void)hipEventDestroy(e);
    prof_collect(c);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    for (auto& kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->staged) (void)hipEventDestroy(c->staged);
    delete c;
    return RPA_OK;
}

int rpa_gsphere(const rpa_cell* cell, const double q[3], double ecut, int32_t* out, int capacity, int* ng_out) {
    if (!cell || !q || !ng_out) return fail(RPA_ERR_INPUT, "NULL argument");
    if (!(ecut >= 0.0) || !std::isfinite(ecut)) return fail(RPA_ERR_INPUT, "bad cutoff");
    double A[3][3], B[3][3];
    std::memcpy(A, cell->A, sizeof(A));
    if (!(std::fabs(det3(A)) > 0)) return fail(RPA_ERR_INPUT, "singular cell");
    reciprocal(A, B);
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    const double gmax = std::sqrt(2.0 * ecut) + qn;
    int mmax[3];
    for (int i = 0; i < 3; ++i) {
        const double al = std::sqrt(A[i][0] * A[i][0] + A[i][1] * A[i][1] + A[i][2] * A[i][2]);
        mmax[i] = (int)std::floor(gmax * al / kTwoPi) + 1;
    }
    struct E {
        double k2;
        int32_t m[3];
    };
    std::vector<E> v;
    for (int a = -mmax[0]; a <= mmax[0]; ++a)
        for (int b = -mmax[1]; b <= mmax[1]; ++b)
            for (int cc = -mmax[2]; cc <= mmax[2]; ++cc) {
                int32_t m[3] = {a, b, cc};
                double k[3];
                const double k2 = kvec(B, q, m, k);
                if (0.5 * k2 <= ecut) v.push_back({k2, {a, b, cc}});
            }
    std::sort(v.begin(), v.end(), [](const E& x, const E& y) {
        if (x.k2 != y.k2) return x.k2 < y.k2;
        if (x.m[0] != y.m[0]) return x.m[0] < y.m[0];
        if (x.m[1] != y.m[1]) return x.m[1] < y.m[1];
        return x.m[2] < y.m[2];
    });
    *ng_out = (int)v.size();
    if (out) {
        if ((int)v.size() > capacity) return fail(RPA_ERR_SHAPE, "capacity too small for the G-sphere");
        for (size_t i = 0; i < v.size(); ++i)
            for (int d = 0; d < 3; ++d) out[3 * i + d] = v[i].m[d];
    }
    return RPA_OK;
}

int rpa_pair_density(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, const rpa_qspec* qs, int npairs,
                     const int32_t* pn, const int32_t* pm, rpa_precision prec, void* rho_out, void* stream) {
    int rc = check_common(c, k, kq, 1, qs);
    if (rc) return rc;
    if (npairs < 0 || (npairs > 0 && (!pn || !pm || !rho_out))) return fail(RPA_ERR_INPUT, "bad pair list");
    Batch B;
    rc = begin(B, c, nullptr, prec, stream);
    if (rc) return rc;
    if (npairs == 0) return check_pair(c, k, kq, qs);
    rc = plan_batch(B, k, kq, 1, qs, 1, false, false, "tables", pn, pm, npairs);
    if (rc) return rc;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        KSet& K = B.ks[0];
        QJob& Q = B.qj[0];
        cplx<T>* phik = nullptr;
        cplx<T>* phikq = nullptr;
        int r = enqueue_unfold(B);
        if (r) return r;
        r = enqueue_orbitals<T>(B, K.k, K.d_mapk, K.zcolk, K.d_zcolk, "phi_k", &phik);
        if (r) return r;
        if (same_set(K.k, K.kq)) phikq = phik;
        else {
            r = enqueue_orbitals<T>(B, K.kq, K.d_mapkq, K.zcolkq, K.d_zcolkq, "phi_kq", &phikq);
            if (r) return r;
        }
        const int NGp = Q.qp.NGp, Pc = Q.Pc;
        T* rre = static_cast<T*>(buf(B, "rho"));
        T* rim = rre + (size_t)Pc * NGp;
        for (int p0 = 0; p0 < npairs; p0 += Pc) {
            const int np = std::min(Pc, npairs - p0);
            r = enqueue_pairs<T>(B, Q, K, 0, phik, phikq, p0, np, rre, rim);
            if (r) return r;
            HIP_TRY(launch_rho_out<T>(rre, rim, np, Q.qp.NG, NGp,
                                      static_cast<double*>(rho_out) + 2 * (size_t)p0 * Q.qp.NG, B.s));
        }
        return RPA_OK;
    };
    return prec == RPA_FP64 ? run(double()) : run(float());
}

static int chi0_impl(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, const rpa_freq* fr,
                     rpa_precision prec, void* chi0_out, int add, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!chi0_out) return fail(RPA_ERR_INPUT, "NULL chi0_out");
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    Batch B;
    rc = begin(B, c, fr, prec, stream);
    if (rc) return rc;
    B.m_major = true;
    rc = plan_batch(B, k, kq, nk, qs, 1, false, true, "tables");
    if (rc) return rc;
    rc = prec == RPA_FP64 ? enqueue_chi0<double>(B) : enqueue_chi0<float>(B);
    if (rc) return rc;
    QJob& Q = B.qj[0];
    HIP_TRY(launch_chi_out(Q.cr, Q.ci, Q.ld, Q.qp.NG, B.nw, add, static_cast<double*>(chi0_out), B.s));
    return RPA_OK;
}

int rpa_chi0(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, const rpa_freq* fr,
             rpa_precision prec, void* chi0_out, void* stream) {
    return chi0_impl(c, k, kq, nk, qs, fr, prec, chi0_out, 0, stream);
}

int rpa_chi0_real(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                  const double* omega, int nw, double eta, rpa_precision prec, void* chi0_out, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!chi0_out) return fail(RPA_ERR_INPUT, "NULL chi0_out");
    if (nw <= 0 || nw > 256 || !omega) return fail(RPA_ERR_INPUT, "need 1 to 256 real frequencies");
    for (int i = 0; i < nw; ++i)
        if (!std::isfinite(omega[i])) return fail(RPA_ERR_INPUT, "non-finite frequency");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(RPA_ERR_INPUT, "eta must be positive");
    Batch B;
    rc = begin(B, c, nullptr, prec, stream);
    if (rc) return rc;
    B.realfreq = true;
    B.eta = eta;
    B.nw_user = nw;
    B.nw = 2 * nw;
    B.om.assign(omega, omega + nw);
    B.ow.assign(nw, 0.0);
    B.m_major = true;
    rc = plan_batch(B, k, kq, nk, qs, 1, false, true, "tables");
    if (rc) return rc;
    rc = prec == RPA_FP64 ? enqueue_chi0<double>(B) : enqueue_chi0<float>(B);
    if (rc) return rc;
    QJob& Q = B.qj[0];
    HIP_TRY(launch_chi_out_real(Q.cr, Q.ci, Q.ld, Q.qp.NG, nw, static_cast<double*>(chi0_out), B.s));
    return RPA_OK;
}

int rpa_chi0_add(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                 const rpa_freq* fr, rpa_precision prec, void* chi0_inout, void* stream) {
    return chi0_impl(c, k, kq, nk, qs, fr, prec, chi0_inout, 1, stream);
}

int rpa_ec_noalloc(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                   const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (!c->scratch) return fail(RPA_ERR_HIP, "device scratch not set up");
    if (c->capturing) return fail(RPA_ERR_INPUT, "context busy");
    // arena mode for the duration of the call: workspaces from the scratch, no profiler events
    struct Arena {
        rpa_ctx* c;
        bool prof;
        explicit Arena(rpa_ctx* c_) : c(c_), prof(c_->prof) {
            c->arena = static_cast<char*>(c->scratch);
            c->arena_cap = kScratchBytes;
            c->arena_off = 0;
            c->abufs.clear();
            c->prof = false;
        }
        ~Arena() {
            c->arena = nullptr;
            c->arena_off = 0;
            c->abufs.clear();
            c->prof = prof;
        }
    } arena(c);
    return rpa_ec(c, k, kq, nk, qs, fr, prec, ec_dev, F_dev, stream);
}

int rpa_ec(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, const rpa_freq* fr,
           rpa_precision prec, double* ec_dev, double* F_dev, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!ec_dev) return fail(RPA_ERR_INPUT, "NULL ec_dev");
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    Batch B;
    rc = begin(B, c, fr, prec, stream);
    if (rc) return rc;
    B.m_major = true;
    rc = plan_batch(B, k, kq, nk, qs, 1, true, false, "tables");
    if (rc) return rc;
    rc = prec == RPA_FP64 ? enqueue_chi0<double>(B) : enqueue_chi0<float>(B);
    if (rc) return rc;
    B.qj[0].ec = ec_dev;
    B.qj[0].F = F_dev;
    rc = enqueue_ec_all(B, false, nullptr);
    if (rc) return rc;
    remember_fail_flags(B);
    return RPA_OK;
}

int rpa_ec_from_chi0(rpa_ctx* c, const rpa_qspec* qs, const rpa_freq* fr, const void* chi0, double* ec_dev,
                     double* F_dev, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (!chi0 || !ec_dev || !qs) return fail(RPA_ERR_INPUT, "NULL chi0, qspec or ec_dev");
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    Batch B;
    int rc = begin(B, c, fr, RPA_FP64, stream);
    if (rc) return rc;
    B.qj.resize(1);
    QJob& Q = B.qj[0];
    Q.qs = qs;
    rc = plan_q(c, qs, Q.qp, true);
    if (rc) return rc;
    Q.ld = Q.qp.NGp;
    B.cls.assign(1, QClass{Q.ld, 0, 1, nullptr, nullptr});
    Upload up;
    up.add(Q.qp.vsqrt, &Q.d_vs);
    up.add(B.ow, &B.d_ow);
    rc = do_upload(c, up, B.s, "tables");
    if (rc) return rc;
    WorkSizes W;
    rc = presize(B, true, false, W);
    if (rc) return rc;
    Q.ec = ec_dev;
    Q.F = F_dev;
    rc = enqueue_ec_all(B, true, chi0);
    if (rc) return rc;
    remember_fail_flags(B);
    return RPA_OK;
}

// E_c of nq q-points in one call; qk (nq + 1 entries, optional): q-point j uses the sets qk[j] .. qk[j+1]-1
// of k and kq (every set for every q-point without it)
static int ec_batched_impl(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, int nq, const rpa_qspec* qs,
                           const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, int use_graph,
                           void* stream, const int* qk) {
    if (nq <= 0 || !qs) return fail(RPA_ERR_INPUT, "need at least one q-point");
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!ec_dev) return fail(RPA_ERR_INPUT, "NULL ec_dev");
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    Batch B;
    rc = begin(B, c, fr, prec, stream);
    if (rc) return rc;
    B.m_major = true;
    uint64_t key = use_graph ? batch_key(k, kq, nk, nq, qs, fr, prec, ec_dev, F_dev, stream) : 0;
    if (use_graph && qk) {
        Fnv h;
        h.val(key);
        h.bytes(qk, sizeof(int) * (size_t)(nq + 1));
        key = h.h;
    }
    if (use_graph && c->graph_exec && c->graph_key == key) {
        HIP_TRY(hipGraphLaunch(c->graph_exec, B.s));
        return RPA_OK;
    }
    if (use_graph) {
        drop_graph(c);
        B.prefix = "g:";
    }
    const std::string tables = B.prefix + "tables";
    rc = plan_batch(B, k, kq, nk, qs, nq, true, false, tables.c_str(), nullptr, nullptr, -1, qk);
    if (rc) return rc;
    std::vector<double> wq(nq);
    for (int j = 0; j < nq; ++j) wq[j] = qs[j].weight;
    auto enqueue_all = [&]() -> int {
        int r = prec == RPA_FP64 ? enqueue_chi0<double>(B) : enqueue_chi0<float>(B);
        if (r) return r;
        for (auto& Q : B.qj) {
            Q.ec = ec_dev + Q.orig;
            Q.F = F_dev ? F_dev + (size_t)Q.orig * B.nw : nullptr;
        }
        r = enqueue_ec_all(B, false, nullptr);
        if (r) return r;
        HIP_TRY(launch_weighted_sum(ec_dev, static_cast<const double*>(B.d_wq), nq, ec_dev + nq, B.s));
        return RPA_OK;
    };
    {
        Upload up;
        up.add(wq, &B.d_wq);
        rc = do_upload(c, up, B.s, (B.prefix + "qweights").c_str());
        if (rc) return rc;
    }
    if (!use_graph) {
        rc = enqueue_all();
        if (rc) return rc;
        remember_fail_flags(B);
        return RPA_OK;
    }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    rc = ensure_lookahead(c);
    if (rc) return rc;
    hipStream_t caller = B.s;
    hipGraph_t graph = nullptr;
    c->capturing = true;
    B.s = c->cap_stream;
    HIP_TRY(hipStreamBeginCapture(B.s, hipStreamCaptureModeThreadLocal));
    rc = enqueue_all();
    hipError_t e = hipStreamEndCapture(B.s, &graph);
    B.s = caller;
    c->capturing = false;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(RPA_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(RPA_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->graph = graph;
    c->graph_exec = exec;
    c->graph_key = key;
    HIP_TRY(hipGraphLaunch(exec, B.s));
    remember_fail_flags(B);
    return RPA_OK;
}


int rpa_ec_batched(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, int nq, const rpa_qspec* qs,
                   const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, int use_graph,
                   void* stream) {
    return ec_batched_impl(c, k, kq, nk, nq, qs, fr, prec, ec_dev, F_dev, use_graph, stream, nullptr);
}

int rpa_ec_batched_sets(rpa_ctx* c, int nq, const rpa_states* const* k, const rpa_states* const* kq, const int* nk,
                        const rpa_qspec* qs, const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev,
                        int use_graph, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (nq <= 0 || !qs || !k || !kq || !nk) return fail(RPA_ERR_INPUT, "need nq > 0 and per-q set lists");
    std::vector<rpa_states> fk, fkq;
    std::vector<int> qk(nq + 1, 0);
    for (int j = 0; j < nq; ++j) {
        if (nk[j] <= 0 || !k[j] || !kq[j])
            return fail(RPA_ERR_INPUT, "q-point " + std::to_string(j) + " has no (k, k+q) state-set pair");
        for (int i = 0; i < nk[j]; ++i) {
            fk.push_back(k[j][i]);
            fkq.push_back(kq[j][i]);
        }
        qk[j + 1] = qk[j] + nk[j];
    }
    return ec_batched_impl(c, fk.data(), fkq.data(), (int)fk.size(), nq, qs, fr, prec, ec_dev, F_dev, use_graph,
                           stream, qk.data());
}

int rpa_ec_backward(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                    const rpa_freq* fr, const double* dEc, double* ec_dev, double* deps_k, void* dC_k, void* dP_k,
                    double* deps_kq, void* dC_kq, void* dP_kq, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!fr || !dEc || !ec_dev || !deps_k || !dC_k) return fail(RPA_ERR_INPUT, "NULL argument");
    if ((long long)c->N[0] * c->N[1] > 16 * 256) return fail(RPA_ERR_UNSUPPORTED, "adjoint needs N1*N2 <= 4096");
    if (fr->nw > 64) return fail(RPA_ERR_UNSUPPORTED, "the adjoint takes at most 64 frequencies");
    // gradient slots: set i of k (of kq) at the sum of the sizes of sets 0 .. i-1 of k (of kq)
    std::vector<BwOut> outk(nk), outkq(nk);
    size_t ek = 0, ck = 0, pk = 0, eq = 0, cq = 0, pq = 0;
    bool any_distinct = false;
    for (int i = 0; i < nk; ++i) {
        if (qs->optical && (k[i].dfde || kq[i].dfde))
            return fail(RPA_ERR_UNSUPPORTED, "the adjoint has no intraband head (state sets with -df/de)");
        if (k[i].sym || kq[i].sym)
            return fail(RPA_ERR_UNSUPPORTED, "the adjoint takes state sets without a symmetry operation");
        const bool same = same_set(&k[i], &kq[i]);
        any_distinct = any_distinct || !same;
        const size_t np = (size_t)(k[i].natoms > 0 ? k[i].proj_off[k[i].natoms] : 0);
        outk[i].deps = deps_k + ek;
        outk[i].dC = static_cast<double*>(dC_k) + ck;
        outk[i].dP = dP_k ? static_cast<double*>(dP_k) + pk : nullptr;
        ek += (size_t)k[i].nbands;
        ck += 2 * (size_t)k[i].nbands * k[i].nQ;
        pk += 2 * (size_t)k[i].nbands * np;
        outkq[i].deps = deps_kq ? deps_kq + eq : nullptr;
        outkq[i].dC = dC_kq ? static_cast<double*>(dC_kq) + cq : nullptr;
        outkq[i].dP = dP_kq ? static_cast<double*>(dP_kq) + pq : nullptr;
        eq += (size_t)kq[i].nbands;
        cq += 2 * (size_t)kq[i].nbands * kq[i].nQ;
        pq += 2 * (size_t)kq[i].nbands * np;
    }
    if (any_distinct && (!deps_kq || !dC_kq)) return fail(RPA_ERR_INPUT, "distinct k+q sets need their own gradient outputs");
    if (k[0].natoms > 0 && (!dP_k || (any_distinct && !dP_kq))) return fail(RPA_ERR_INPUT, "NULL projection gradient");
    Batch B;
    rc = begin(B, c, fr, RPA_FP64, stream);
    if (rc) return rc;
    B.allow_paw_mfma = false;
    rc = plan_batch(B, k, kq, nk, qs, 1, true, false, "tables");
    if (rc) return rc;
    size_t total = 0;
    for (auto& K : B.ks) total += K.pn.size();
    if (total == 0) return fail(RPA_ERR_INPUT, "no transitions (f_n - f_m > 1e-8) in the state sets");
    return backward(B, dEc, ec_dev, outk, outkq);
}

int rpa_set_pair_path(rpa_ctx* ctx, int path) {
    if (!ctx) return fail(RPA_ERR_INPUT, "NULL context");
    if (path != 0 && path != 1) return fail(RPA_ERR_INPUT, "pair path must be 0 or 1");
    if (ctx->pair_reg != (path == 0)) drop_graph(ctx);
    ctx->pair_reg = path == 0;
    return RPA_OK;
}

int rpa_set_chunk_pairs(rpa_ctx* ctx, int max_pairs) {
    if (!ctx) return fail(RPA_ERR_INPUT, "NULL context");
    if (max_pairs < 0) return fail(RPA_ERR_INPUT, "chunk bound must be >= 0");
    if (ctx->max_chunk != max_pairs) drop_graph(ctx);
    ctx->max_chunk = max_pairs;
    return RPA_OK;
}

int rpa_set_paw_window(rpa_ctx* ctx, int max_bands) {
    if (!ctx) return fail(RPA_ERR_INPUT, "NULL context");
    if (max_bands < 0) return fail(RPA_ERR_INPUT, "PAW window bound must be >= 0");
    if (ctx->paw_win != max_bands) drop_graph(ctx);
    ctx->paw_win = max_bands;
    return RPA_OK;
}

int rpa_tune_set(rpa_ctx* c, rpa_precision prec, int NG, int variant) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (prec == RPA_FP64) return variant == 0 ? RPA_OK : fail(RPA_ERR_INPUT, "FP64 has one kernel variant (0)");
    if (variant != 1 && variant != 4 && variant != 5)
        return fail(RPA_ERR_INPUT, "split variants are 1 (64x64), 4 (64x128 pipelined, FP64 accumulation) and 5 "
                                   "(as 4, eight waves)");
    const int NGp = (NG + kTile - 1) / kTile * kTile;
    c->tune[tune_key(prec, NGp)] = variant;
    return RPA_OK;
}

int rpa_tune_get(rpa_ctx* c, rpa_precision prec, int NG, int* variant) {
    if (!c || !variant) return fail(RPA_ERR_INPUT, "NULL argument");
    *variant = default_variant(c, prec, (NG + kTile - 1) / kTile * kTile);
    return RPA_OK;
}

int rpa_autotune(rpa_ctx* c, rpa_precision prec, int NG, int npairs, int nw, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (prec == RPA_FP64) return RPA_OK;
    if (NG <= 0 || npairs <= 0 || nw <= 0) return fail(RPA_ERR_INPUT, "bad tuning shape");
    HIP_TRY(hipSetDevice(c->device));
    return autotune_run(c, prec, NG, npairs, nw, static_cast<hipStream_t>(stream));
}

int rpa_set_autotune(rpa_ctx* c, int enable) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    c->autotune = enable != 0;
    return RPA_OK;
}

}  // extern "C"

namespace {

// Time the split rank-k variants on synthetic operands of one shape (stream-ordered, synchronizes) and record
// the fastest for the padded sphere of NG.
int autotune_run(rpa_ctx* c, rpa_precision prec, int NG, int npairs, int nw, hipStream_t s) {
    const int NGp = (NG + kTile - 1) / kTile * kTile;
    Batch B;
    B.c = c;
    B.s = s;
    B.prec = prec;
    B.nw = nw;
    B.prefix = "tune:";
    B.ld = NGp;
    B.qj.resize(1);
    QJob& Q = B.qj[0];
    Q.qp.NG = NG;
    Q.qp.NGp = NGp;
    Q.ld = NGp;
    const int lda = (npairs + 3) / 4 * 4;
    const int NGq = (NGp + 127) / 128 * 128;
    const size_t blk = (size_t)((npairs + 31) / 32) * NGq * 32;
    void *rho, *aw, *chi, *pack, *sc;
    int rc = get_buf(c, "tune:rho", 2 * (size_t)npairs * NGp * sizeof(float), s, &rho);
    if (!rc) rc = get_buf(c, "tune:weights", (size_t)nw * lda * sizeof(double), s, &aw);
    if (!rc) rc = get_buf(c, "tune:chi", 2 * (size_t)nw * NGp * NGp * sizeof(double), s, &chi);
    if (!rc) rc = get_buf(c, "tune:split_pack", blk * (2 * sizeof(float) + 4 * sizeof(unsigned short)), s, &pack);
    if (!rc) rc = get_buf(c, "tune:split_scales", (size_t)(nw + 1 + 256) * sizeof(float), s, &sc);
    if (rc) return rc;
    HIP_TRY(launch_fill_pattern(static_cast<float*>(rho), 2 * (size_t)npairs * NGp, static_cast<double*>(aw),
                                (size_t)nw * lda, s));
    Q.cr = static_cast<double*>(chi);
    Q.ci = Q.cr + (size_t)nw * NGp * NGp;
    const float* rre = static_cast<const float*>(rho);
    const float* rim = rre + (size_t)npairs * NGp;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e300;
    int bestv = 1;
    // each variant on the same operands, compared by time per pair
    for (int v : {1, 4, 5}) {
        Q.variant = v;
        const int kv = npairs;
        double tmin = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipEventRecord(e0, s));
            rc = enqueue_update<float>(B, Q, kv, rre, rim, static_cast<const double*>(aw), lda);
            if (rc) break;
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tmin = std::min(tmin, (double)ms / kv * npairs);
        }
        if (rc) break;
        if (tmin < best) {
            best = tmin;
            bestv = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    c->tune[tune_key(prec, NGp)] = bestv;
    c->tune_ms[tune_key(prec, NGp)] = best;
    return RPA_OK;
}

}  // namespace

extern "C" {

int rpa_tune_cache_io(rpa_ctx* c, const char* path, int save) {
    if (!c || !path) return fail(RPA_ERR_INPUT, "NULL argument");
    if (save) {
        FILE* f = std::fopen(path, "w");
        if (!f) return fail(RPA_ERR_INPUT, std::string("cannot write ") + path);
        std::fprintf(f, "# precision padded_NG variant (1 = 64x64, 4 / 5 = pipelined 64x128)\n");
        for (auto& kv : c->tune) std::fprintf(f, "%d %d %d\n", (int)(kv.first >> 32), (int)(kv.first & 0xffffffff), kv.second);
        std::fclose(f);
        return RPA_OK;
    }
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(RPA_ERR_INPUT, std::string("cannot read ") + path);
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#') continue;
        int p, ng, v;
        if (std::sscanf(line, "%d %d %d", &p, &ng, &v) == 3 && (v == 1 || v == 4 || v == 5) && ng > 0)
            c->tune[tune_key((rpa_precision)p, ng)] = v;
    }
    std::fclose(f);
    return RPA_OK;
}

int rpa_profile(rpa_ctx* c, int enable) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    HIP_TRY(hipSetDevice(c->device));
    prof_collect(c);
    for (int i = 0; i < S_COUNT; ++i) {
        c->prof_ms[i] = 0;
        c->prof_n[i] = 0;
    }
    c->prof = enable != 0;
    return RPA_OK;
}

int rpa_profile_get(rpa_ctx* c, const char* stage, double* ms, long long* launches) {
    if (!c || !stage || !ms || !launches) return fail(RPA_ERR_INPUT, "NULL argument");
    HIP_TRY(hipSetDevice(c->device));
    prof_collect(c);
    for (int i = 0; i < S_COUNT; ++i)
        if (std::strcmp(stage, kStageNames[i]) == 0) {
            *ms = c->prof_ms[i];
            *launches = c->prof_n[i];
            return RPA_OK;
        }
    return fail(RPA_ERR_INPUT, std::string("unknown stage ") + stage);
}

int rpa_check(rpa_ctx* c, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(hipGetLastError());
    if (!c->last_fail || c->last_nw <= 0) return RPA_OK;
    const int n = c->last_nw * std::max(c->last_nq, 1);
    std::vector<int> f(n);
    HIP_TRY(hipMemcpy(f.data(), c->last_fail, sizeof(int) * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i)
        if (f[i])
            return fail(RPA_ERR_NOT_PD, "1 - K not positive definite at q index " +
                                            std::to_string((size_t)(i / c->last_nw) < c->last_qorder.size()
                                                               ? c->last_qorder[i / c->last_nw]
                                                               : i / c->last_nw) +
                                            ", frequency index " + std::to_string(i % c->last_nw) + " (pivot " +
                                            std::to_string(f[i] - 1) + ")");
    return RPA_OK;
}

}  // extern "C"
