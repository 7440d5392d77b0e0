// Host runtime behind the C ABI of include/rpa.h: validation, G-sphere and
// index tables, pair lists, workspace management and the launch sequence of
// Table 1 steps 3-13 (orbitals, pair densities, PAW, optical row, weights,
// grouped rank-k update, Cholesky log-determinant, frequency sum).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
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
};

namespace {

// ---------------------------------------------------------------- profiler
enum Stage { S_ORB = 0, S_PAIR_XY, S_PAIR_Z, S_PAW, S_OPTICAL, S_WEIGHTS, S_HERK, S_CHOL, S_OTHER, S_COUNT };
const char* kStageNames[S_COUNT] = {"orbitals", "pair_xy", "pair_z_gather", "paw", "optical", "weights",
                                    "herk", "cholesky", "other"};

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
        if (c->prof && (a = prof_event(c))) (void)hipEventRecord(a, s);
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

// ---------------------------------------------------------------- buffers
int get_buf(rpa_ctx* c, const char* name, size_t bytes, hipStream_t s, void** out) {
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

int do_upload(rpa_ctx* c, Upload& u, hipStream_t s) {
    if (u.total == 0) return RPA_OK;
    if (c->staged_valid) HIP_TRY(hipEventSynchronize(c->staged));
    if (c->pinned_bytes < u.total) {
        if (c->pinned) HIP_TRY(hipHostFree(c->pinned));
        c->pinned = nullptr;
        c->pinned_bytes = 0;
        HIP_TRY(hipHostMalloc(&c->pinned, u.total, hipHostMallocDefault));
        c->pinned_bytes = u.total;
    }
    void* dev = nullptr;
    int rc = get_buf(c, "tables", u.total, s, &dev);
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
    std::vector<double> vsqrt;
};

int plan_q(rpa_ctx* c, const rpa_qspec* qs, QPlan& P, bool need_coulomb) {
    if (!qs) return fail(RPA_ERR_INPUT, "NULL qspec");
    if (qs->NG <= 0 || !qs->gmiller) return fail(RPA_ERR_SHAPE, "empty G-sphere");
    const int NG = qs->NG;
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = hi[d] = qs->gmiller[d];
    }
    for (int i = 0; i < NG; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], (int)qs->gmiller[3 * i + d]);
            hi[d] = std::max(hi[d], (int)qs->gmiller[3 * i + d]);
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

void pair_list(const rpa_states* k, const rpa_states* kq, std::vector<int32_t>& pn, std::vector<int32_t>& pm) {
    pn.clear();
    pm.clear();
    for (int n = 0; n < k->nbands; ++n)
        for (int m = 0; m < kq->nbands; ++m)
            if (k->f[n] - kq->f[m] > kDeltaF) {
                pn.push_back(n);
                pm.push_back(m);
            }
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
    std::vector<cplx<T>> t(N);
    for (int i = 0; i < N; ++i) {
        const double a = kTwoPi * i / N;
        t[i] = mk(T(std::cos(a)), T(-std::sin(a)));
    }
    return t;
}

// ------------------------------------------------------------ the engine
struct Engine {
    rpa_ctx* c;
    hipStream_t s;
    rpa_precision prec;
    const rpa_qspec* qs;
    QPlan qp;
    int nw = 0;

    // device table pointers
    void* d_kx = nullptr; void* d_ky = nullptr; void* d_cs = nullptr; void* d_cg = nullptr; void* d_ckz = nullptr;
    void* d_vs = nullptr; void* d_om = nullptr; void* d_ow = nullptr;
    void* d_tw[3] = {nullptr, nullptr, nullptr};
    void* d_qoff = nullptr; void* d_poff = nullptr;

    // host tables kept alive until upload
    std::vector<int32_t> qoff, poff;
    std::vector<double> om, ow;
    std::vector<cplx<double>> tw64[3];
    std::vector<cplx<float>> tw32[3];

    bool fp64() const { return prec == RPA_FP64; }
};

struct KSet {
    const rpa_states* k;
    const rpa_states* kq;
    std::vector<int32_t> pn, pm;
    std::vector<int32_t> mapk, mapkq;
    std::vector<double> epsk, epskq, fk, fkq;
    std::vector<double> wq, Dq;
    void* d_pn = nullptr; void* d_pm = nullptr;
    void* d_mapk = nullptr; void* d_mapkq = nullptr;
    void* d_epsk = nullptr; void* d_epskq = nullptr; void* d_fk = nullptr; void* d_fkq = nullptr;
    void* d_wq = nullptr; void* d_Dq = nullptr;
    std::vector<int32_t> nlist_all;  // n = 0 .. nbands-1
    void* d_nlist = nullptr;
};

int chunk_size(const Engine& E, size_t elem) {
    const PairGeom& g = E.qp.g;
    const size_t per = (size_t)g.N3 * g.ncols * 2 * elem + 2 * (size_t)g.NGp * elem + (size_t)E.nw * 8;
    size_t budget = (size_t)6 << 30;
    if (E.c->cap) budget = std::min(budget, E.c->cap / 3);
    size_t pc = budget / per;
    pc = std::max<size_t>(pc, 64);
    pc = std::min<size_t>(pc, 1 << 20);
    return (int)pc;
}

template <typename T>
int run_orbitals(Engine& E, const rpa_states* s, void* d_map, const char* name, cplx<T>** out) {
    rpa_ctx* c = E.c;
    const size_t vol = (size_t)c->N[0] * c->N[1] * c->N[2];
    void* p = nullptr;
    int rc = get_buf(c, name, (size_t)s->nbands * vol * sizeof(cplx<T>), E.s, &p);
    if (rc) return rc;
    cplx<T>* phi = static_cast<cplx<T>*>(p);
    ProfScope ps_(c, S_ORB, E.s);
    HIP_TRY(launch_fill_zero<T>(phi, (size_t)s->nbands * vol, E.s));
    HIP_TRY(launch_orb_scatter<T>(static_cast<const double*>(s->C), s->nbands, s->nQ,
                                  static_cast<const int32_t*>(d_map), vol, phi, E.s));
    for (int ax = 0; ax < 3; ++ax)
        HIP_TRY(launch_fft_axis<T>(phi, s->nbands, c->N[0], c->N[1], c->N[2], ax, c->plan[ax],
                                   static_cast<const cplx<T>*>(E.d_tw[ax]), +1, E.s));
    *out = phi;
    return RPA_OK;
}

int prepare_common(Engine& E, Upload& up) {
    rpa_ctx* c = E.c;
    const QPlan& q = E.qp;
    up.add(q.kx, &E.d_kx);
    up.add(q.ky, &E.d_ky);
    up.add(q.col_start, &E.d_cs);
    up.add(q.col_g, &E.d_cg);
    up.add(q.col_kz, &E.d_ckz);
    up.add(q.vsqrt, &E.d_vs);
    up.add(E.om, &E.d_om);
    up.add(E.ow, &E.d_ow);
    for (int ax = 0; ax < 3; ++ax) {
        if (E.fp64()) {
            E.tw64[ax] = twiddles<double>(c->N[ax]);
            up.add(E.tw64[ax], &E.d_tw[ax]);
        } else {
            E.tw32[ax] = twiddles<float>(c->N[ax]);
            up.add(E.tw32[ax], &E.d_tw[ax]);
        }
    }
    return RPA_OK;
}

int prepare_kset(Engine& E, KSet& K, Upload& up, bool need_pairs_from_f, const int32_t* pn_in = nullptr,
                 const int32_t* pm_in = nullptr, int np_in = 0) {
    const rpa_states* k = K.k;
    const rpa_states* kq = K.kq;
    if (need_pairs_from_f) {
        pair_list(k, kq, K.pn, K.pm);
    } else {
        K.pn.assign(pn_in, pn_in + np_in);
        K.pm.assign(pm_in, pm_in + np_in);
        for (int i = 0; i < np_in; ++i)
            if (K.pn[i] < 0 || K.pn[i] >= k->nbands || K.pm[i] < 0 || K.pm[i] >= kq->nbands)
                return fail(RPA_ERR_SHAPE, "pair index out of range");
    }
    K.mapk = scatter_map(E.c, k);
    up.add(K.pn, &K.d_pn);
    up.add(K.pm, &K.d_pm);
    up.add(K.mapk, &K.d_mapk);
    if (!same_set(k, kq)) {
        K.mapkq = scatter_map(E.c, kq);
        up.add(K.mapkq, &K.d_mapkq);
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
    if (E.qs->optical) {
        double B[3][3];
        std::memcpy(B, E.c->B, sizeof(B));
        K.wq.resize(k->nQ);
        double qh[3] = {E.qs->qhat[0], E.qs->qhat[1], E.qs->qhat[2]};
        const double nrm = std::sqrt(qh[0] * qh[0] + qh[1] * qh[1] + qh[2] * qh[2]);
        if (!(nrm > 0)) return fail(RPA_ERR_INPUT, "optical limit needs a nonzero qhat");
        for (int d = 0; d < 3; ++d) qh[d] /= nrm;
        for (int i = 0; i < k->nQ; ++i) {
            double kv[3];
            kvec(B, k->kpt, k->miller + 3 * i, kv);
            K.wq[i] = qh[0] * kv[0] + qh[1] * kv[1] + qh[2] * kv[2];
        }
        up.add(K.wq, &K.d_wq);
        const int nq2 = (int)E.qoff.back();
        K.Dq.assign(std::max(nq2, 1), 0.0);
        if (nq2 > 0)
            for (int e = 0; e < nq2; ++e)
                K.Dq[e] = qh[0] * E.qs->Dpaw[e] + qh[1] * E.qs->Dpaw[nq2 + e] + qh[2] * E.qs->Dpaw[2 * nq2 + e];
        up.add(K.Dq, &K.d_Dq);
    }
    return RPA_OK;
}

// rho for pairs [p0, p0 + np) of K into planar buffers rre/rim [np][NGp]
template <typename T>
int pair_chunk(Engine& E, KSet& K, const cplx<T>* phik, const cplx<T>* phikq, int p0, int np, T* rre, T* rim) {
    rpa_ctx* c = E.c;
    const PairGeom& g = E.qp.g;
    void* tb = nullptr;
    int rc = get_buf(c, "tbuf", (size_t)np * g.N3 * g.ncols * sizeof(cplx<T>), E.s, &tb);
    if (rc) return rc;
    const int32_t* pn = static_cast<const int32_t*>(K.d_pn) + p0;
    const int32_t* pm = static_cast<const int32_t*>(K.d_pm) + p0;
    {
    ProfScope ps_(c, S_PAIR_XY, E.s);
    HIP_TRY(launch_pair_xy<T>(phik, phikq, pn, pm, np, g, static_cast<const int32_t*>(E.d_kx),
                              static_cast<const int32_t*>(E.d_ky), static_cast<const cplx<T>*>(E.d_tw[0]),
                              static_cast<const cplx<T>*>(E.d_tw[1]), static_cast<cplx<T>*>(tb), E.s));
    }
    {
    ProfScope ps_(c, S_PAIR_Z, E.s);
    HIP_TRY(launch_pair_z_gather<T>(static_cast<const cplx<T>*>(tb), np, g, static_cast<const int32_t*>(E.d_cs),
                                    static_cast<const int32_t*>(E.d_cg), static_cast<const int32_t*>(E.d_ckz),
                                    static_cast<const cplx<T>*>(E.d_tw[2]), rre, rim, E.s));
    }
    const int nproj = nproj_total(K.k);
    if (nproj > 0) {
        // Y for the band window [nlo, nhi] of this chunk
        int nlo = K.pn[p0], nhi = K.pn[p0];
        for (int i = p0; i < p0 + np; ++i) {
            nlo = std::min(nlo, (int)K.pn[i]);
            nhi = std::max(nhi, (int)K.pn[i]);
        }
        const int nn = nhi - nlo + 1;
        void* y = nullptr;
        rc = get_buf(c, "paw_y", 2 * (size_t)nn * nproj * g.NGp * sizeof(T), E.s, &y);
        if (rc) return rc;
        T* Yre = static_cast<T*>(y);
        T* Yim = Yre + (size_t)nn * nproj * g.NGp;
        ProfScope ps_(c, S_PAW, E.s);
        HIP_TRY(launch_paw_y<T>(static_cast<const double*>(K.k->P), nproj, static_cast<const int32_t*>(K.d_nlist) + nlo,
                                nn, static_cast<const int32_t*>(E.d_poff), static_cast<const int32_t*>(E.d_qoff),
                                K.k->natoms, nproj, static_cast<const double*>(E.qs->Qpaw), g.NG, g.NGp, Yre, Yim,
                                E.s));
        HIP_TRY(launch_paw_add<T>(Yre, Yim, pn, nlo, pm, static_cast<const double*>(K.kq->P), nproj, nproj, np, g.NG,
                                  g.NGp, rre, rim, E.s));
    }
    if (E.qs->optical && E.qp.g0 >= 0) {
        ProfScope ps_(c, S_OPTICAL, E.s);
        HIP_TRY(launch_optical_row<T>(static_cast<const double*>(K.k->C), static_cast<const double*>(K.kq->C), K.k->nQ,
                                      static_cast<const double*>(K.d_wq), static_cast<const double*>(K.k->P),
                                      static_cast<const double*>(K.kq->P), nproj, static_cast<const double*>(K.d_Dq),
                                      static_cast<const int32_t*>(E.d_poff), static_cast<const int32_t*>(E.d_qoff),
                                      K.k->natoms, static_cast<const double*>(K.d_epsk),
                                      static_cast<const double*>(K.d_epskq), pn, pm, np, E.qp.g0, g.NGp, rre, rim,
                                      E.s));
    }
    return RPA_OK;
}

int begin(Engine& E, rpa_ctx* c, const rpa_qspec* qs, const rpa_freq* fr, rpa_precision prec, void* stream) {
    E.c = c;
    E.s = static_cast<hipStream_t>(stream);
    E.prec = prec;
    E.qs = qs;
    if (prec != RPA_FP64 && prec != RPA_SPLIT_BF16 && prec != RPA_SPLIT_FP16)
        return fail(RPA_ERR_INPUT, "unknown precision");
    HIP_TRY(hipSetDevice(c->device));
    int rc = plan_q(c, qs, E.qp, fr != nullptr);
    if (rc) return rc;
    if (fr) {
        rc = check_freq(fr);
        if (rc) return rc;
        E.nw = fr->nw;
        E.om.assign(fr->omega, fr->omega + fr->nw);
        E.ow.assign(fr->weight, fr->weight + fr->nw);
    }
    return RPA_OK;
}

int set_paw_tables(Engine& E, const rpa_states* k, Upload& up) {
    const int na = k->natoms;
    E.poff.assign(na + 1, 0);
    E.qoff.assign(na + 1, 0);
    for (int a = 0; a <= na && na > 0; ++a) E.poff[a] = k->proj_off[a];
    for (int a = 0; a < na; ++a) {
        const int np = k->proj_off[a + 1] - k->proj_off[a];
        E.qoff[a + 1] = E.qoff[a] + np * np;
    }
    up.add(E.poff, &E.d_poff);
    up.add(E.qoff, &E.d_qoff);
    return RPA_OK;
}

// accumulate chi0 (planar, lower tiles) over all k pairs into "chi" buffers
template <typename T>
int accumulate_chi0(Engine& E, const rpa_states* ks, const rpa_states* kqs, int nk, double** chiRe, double** chiIm) {
    rpa_ctx* c = E.c;
    const PairGeom& g = E.qp.g;
    const int NGp = g.NGp;
    std::vector<KSet> sets(nk);
    Upload up;
    int rc = prepare_common(E, up);
    if (rc) return rc;
    rc = set_paw_tables(E, &ks[0], up);
    if (rc) return rc;
    for (int i = 0; i < nk; ++i) {
        sets[i].k = &ks[i];
        sets[i].kq = &kqs[i];
        rc = check_pair(c, &ks[i], &kqs[i], E.qs);
        if (rc) return rc;
        rc = prepare_kset(E, sets[i], up, true);
        if (rc) return rc;
    }
    rc = do_upload(c, up, E.s);
    if (rc) return rc;

    void* chi = nullptr;
    const size_t mat = (size_t)E.nw * NGp * NGp;
    rc = get_buf(c, "chi", 2 * mat * sizeof(double), E.s, &chi);
    if (rc) return rc;
    double* cr = static_cast<double*>(chi);
    double* ci = cr + mat;
    HIP_TRY(launch_fill_zero<double>(reinterpret_cast<cplx<double>*>(cr), mat, E.s));

    for (int i = 0; i < nk; ++i) {
        KSet& K = sets[i];
        const int P = (int)K.pn.size();
        if (P == 0) continue;
        cplx<T>* phik = nullptr;
        cplx<T>* phikq = nullptr;
        rc = run_orbitals<T>(E, K.k, K.d_mapk, "phi_k", &phik);
        if (rc) return rc;
        if (same_set(K.k, K.kq)) {
            phikq = phik;
        } else {
            rc = run_orbitals<T>(E, K.kq, K.d_mapkq, "phi_kq", &phikq);
            if (rc) return rc;
        }
        const int Pc = std::min(P, chunk_size(E, sizeof(T)));
        const int lda = (Pc + 3) / 4 * 4;
        void* rho = nullptr;
        rc = get_buf(c, "rho", 2 * (size_t)Pc * NGp * sizeof(T), E.s, &rho);
        if (rc) return rc;
        T* rre = static_cast<T*>(rho);
        T* rim = rre + (size_t)Pc * NGp;
        void* aw = nullptr;
        rc = get_buf(c, "weights", (size_t)E.nw * lda * sizeof(double), E.s, &aw);
        if (rc) return rc;
        const double prefac = K.k->weight / c->volume;
        for (int p0 = 0; p0 < P; p0 += Pc) {
            const int np = std::min(Pc, P - p0);
            rc = pair_chunk<T>(E, K, phik, phikq, p0, np, rre, rim);
            if (rc) return rc;
            {
            ProfScope ps_(c, S_WEIGHTS, E.s);
            HIP_TRY(launch_weights(static_cast<const double*>(K.d_epsk), static_cast<const double*>(K.d_epskq),
                                   static_cast<const double*>(K.d_fk), static_cast<const double*>(K.d_fkq),
                                   static_cast<const int32_t*>(K.d_pn) + p0, static_cast<const int32_t*>(K.d_pm) + p0,
                                   np, static_cast<const double*>(E.d_om), E.nw, prefac, static_cast<double*>(aw),
                                   lda, E.s));
            }
            ProfScope ps_(c, S_HERK, E.s);
            if constexpr (sizeof(T) == 8) {
                HerkArgs h{};
                h.Are = reinterpret_cast<const double*>(rre);
                h.Aim = reinterpret_cast<const double*>(rim);
                h.sA = 0;
                h.ldA = NGp;
                h.colA = 0;
                h.K = np;
                h.w = static_cast<const double*>(aw);
                h.sw = lda;
                h.alpha = 0;
                h.Cre = cr;
                h.Cim = ci;
                h.sC = (long long)NGp * NGp;
                h.ldC = NGp;
                h.r0 = 0;
                h.nT = NGp / kTile;
                h.nbatch = E.nw;
                HIP_TRY(launch_herk_f64(h, E.s));
            } else {
                HerkSplitArgs h{};
                h.Are = reinterpret_cast<const float*>(rre);
                h.Aim = reinterpret_cast<const float*>(rim);
                h.ldA = NGp;
                h.K = np;
                h.w = static_cast<const double*>(aw);
                h.lda = lda;
                h.Cre = cr;
                h.Cim = ci;
                h.sC = (long long)NGp * NGp;
                h.ldC = NGp;
                h.nT = NGp / kTile;
                h.nw = E.nw;
                h.fp16 = E.prec == RPA_SPLIT_FP16;
                h.wscale = nullptr;
                HIP_TRY(launch_herk_split(h, E.s));
            }
        }
    }
    *chiRe = cr;
    *chiIm = ci;
    return RPA_OK;
}

// E_c from the planar lower-triangular chi0 accumulator (overwritten)
int ec_stage(Engine& E, double* cr, double* ci, double* ec_dev, double* F_dev, bool from_full, const void* chi_full) {
    rpa_ctx* c = E.c;
    const int NG = E.qp.NG, NGp = E.qp.NGp, nw = E.nw;
    void* sm = nullptr;
    int rc = get_buf(c, "ec_small", (size_t)nw * (2 * sizeof(double) + sizeof(int)) + 64, E.s, &sm);
    if (rc) return rc;
    double* logdet = static_cast<double*>(sm);
    double* trk = logdet + nw;
    int* failv = reinterpret_cast<int*>(trk + nw);
    void* lb = nullptr;
    rc = get_buf(c, "chol_L", 2 * (size_t)nw * kTile * kTile * sizeof(double), E.s, &lb);
    if (rc) return rc;
    double* Lre = static_cast<double*>(lb);
    double* Lim = Lre + (size_t)nw * kTile * kTile;
    void* pb = nullptr;
    rc = get_buf(c, "chol_panel", 2 * (size_t)nw * kTile * NGp * sizeof(double), E.s, &pb);
    if (rc) return rc;
    double* Pre = static_cast<double*>(pb);
    double* Pim = Pre + (size_t)nw * kTile * NGp;
    ProfScope ps_(c, S_CHOL, E.s);
    HIP_TRY(launch_zero(logdet, 2 * nw, failv, nw, E.s));
    if (from_full) {
        HIP_TRY(launch_build_negk_from_full(static_cast<const double*>(chi_full), NG, cr, ci, NGp, nw,
                                            static_cast<const double*>(E.d_vs), trk, E.s));
    } else {
        HIP_TRY(launch_build_negk(cr, ci, NGp, NG, NGp, nw, static_cast<const double*>(E.d_vs), trk, E.s));
    }
    for (int j0 = 0; j0 < NGp; j0 += kTile) {
        HIP_TRY(launch_chol_panel(cr, ci, NGp, j0, nw, Lre, Lim, logdet, failv, E.s));
        const int r0 = j0 + kTile;
        if (r0 >= NGp) break;
        HIP_TRY(launch_chol_trsm(cr, ci, NGp, j0, NGp, nw, Lre, Lim, Pre, Pim, E.s));
        HerkArgs h{};
        h.Are = Pre;
        h.Aim = Pim;
        h.sA = (long long)kTile * NGp;
        h.ldA = NGp;
        h.colA = r0;
        h.K = kTile;
        h.w = nullptr;
        h.sw = 0;
        h.alpha = -1.0;
        h.Cre = cr;
        h.Cim = ci;
        h.sC = (long long)NGp * NGp;
        h.ldC = NGp;
        h.r0 = r0;
        h.nT = (NGp - r0) / kTile;
        h.nbatch = nw;
        HIP_TRY(launch_herk_f64(h, E.s));
    }
    HIP_TRY(launch_finalize(logdet, trk, failv, static_cast<const double*>(E.d_ow), nw, F_dev, ec_dev, E.s));
    c->last_fail = failv;
    c->last_nw = nw;
    return RPA_OK;
}

int check_common(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs) {
    if (!ctx) return fail(RPA_ERR_INPUT, "NULL context");
    if (nk <= 0 || !k || !kq) return fail(RPA_ERR_INPUT, "need at least one (k, k+q) state-set pair");
    if (!qs) return fail(RPA_ERR_INPUT, "NULL qspec");
    for (int i = 1; i < nk; ++i)
        if (k[i].natoms != k[0].natoms) return fail(RPA_ERR_SHAPE, "atom count differs between k-points");
    return RPA_OK;
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
    *out = c;
    return RPA_OK;
}

int rpa_destroy(rpa_ctx* c) {
    if (!c) return RPA_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
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
    Engine E;
    rc = begin(E, c, qs, nullptr, prec, stream);
    if (rc) return rc;
    rc = check_pair(c, k, kq, qs);
    if (rc) return rc;
    if (npairs == 0) return RPA_OK;
    Upload up;
    KSet K;
    K.k = k;
    K.kq = kq;
    prepare_common(E, up);
    set_paw_tables(E, k, up);
    rc = prepare_kset(E, K, up, false, pn, pm, npairs);
    if (rc) return rc;
    // the PAW band window of a chunk is [min n, max n]; keep pairs n-sorted per chunk
    rc = do_upload(c, up, E.s);
    if (rc) return rc;
    auto run = [&](auto tag) -> int {
        using T = decltype(tag);
        cplx<T>* phik = nullptr;
        cplx<T>* phikq = nullptr;
        int r = run_orbitals<T>(E, k, K.d_mapk, "phi_k", &phik);
        if (r) return r;
        if (same_set(k, kq)) phikq = phik;
        else {
            r = run_orbitals<T>(E, kq, K.d_mapkq, "phi_kq", &phikq);
            if (r) return r;
        }
        const int NGp = E.qp.NGp;
        const int Pc = std::min(npairs, chunk_size(E, sizeof(T)));
        void* rho = nullptr;
        r = get_buf(c, "rho", 2 * (size_t)Pc * NGp * sizeof(T), E.s, &rho);
        if (r) return r;
        T* rre = static_cast<T*>(rho);
        T* rim = rre + (size_t)Pc * NGp;
        for (int p0 = 0; p0 < npairs; p0 += Pc) {
            const int np = std::min(Pc, npairs - p0);
            r = pair_chunk<T>(E, K, phik, phikq, p0, np, rre, rim);
            if (r) return r;
            HIP_TRY(launch_rho_out<T>(rre, rim, np, E.qp.NG, NGp, static_cast<double*>(rho_out) + 2 * (size_t)p0 * E.qp.NG,
                                      E.s));
        }
        return RPA_OK;
    };
    return prec == RPA_FP64 ? run(double()) : run(float());
}

int rpa_chi0(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, const rpa_freq* fr,
             rpa_precision prec, void* chi0_out, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!chi0_out) return fail(RPA_ERR_INPUT, "NULL chi0_out");
    Engine E;
    rc = begin(E, c, qs, fr, prec, stream);
    if (rc) return rc;
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    double *cr = nullptr, *ci = nullptr;
    rc = prec == RPA_FP64 ? accumulate_chi0<double>(E, k, kq, nk, &cr, &ci)
                          : accumulate_chi0<float>(E, k, kq, nk, &cr, &ci);
    if (rc) return rc;
    HIP_TRY(launch_chi_out(cr, ci, E.qp.NGp, E.qp.NG, E.nw, static_cast<double*>(chi0_out), E.s));
    return RPA_OK;
}

int rpa_ec(rpa_ctx* c, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs, const rpa_freq* fr,
           rpa_precision prec, double* ec_dev, double* F_dev, void* stream) {
    int rc = check_common(c, k, kq, nk, qs);
    if (rc) return rc;
    if (!ec_dev) return fail(RPA_ERR_INPUT, "NULL ec_dev");
    Engine E;
    rc = begin(E, c, qs, fr, prec, stream);
    if (rc) return rc;
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    double *cr = nullptr, *ci = nullptr;
    rc = prec == RPA_FP64 ? accumulate_chi0<double>(E, k, kq, nk, &cr, &ci)
                          : accumulate_chi0<float>(E, k, kq, nk, &cr, &ci);
    if (rc) return rc;
    return ec_stage(E, cr, ci, ec_dev, F_dev, false, nullptr);
}

int rpa_ec_from_chi0(rpa_ctx* c, const rpa_qspec* qs, const rpa_freq* fr, const void* chi0, double* ec_dev,
                     double* F_dev, void* stream) {
    if (!c) return fail(RPA_ERR_INPUT, "NULL context");
    if (!chi0 || !ec_dev) return fail(RPA_ERR_INPUT, "NULL chi0 or ec_dev");
    Engine E;
    int rc = begin(E, c, qs, fr, RPA_FP64, stream);
    if (rc) return rc;
    if (!fr) return fail(RPA_ERR_INPUT, "NULL frequency grid");
    Upload up;
    up.add(E.qp.vsqrt, &E.d_vs);
    up.add(E.ow, &E.d_ow);
    rc = do_upload(c, up, E.s);
    if (rc) return rc;
    void* chi = nullptr;
    const size_t mat = (size_t)E.nw * E.qp.NGp * E.qp.NGp;
    rc = get_buf(c, "chi", 2 * mat * sizeof(double), E.s, &chi);
    if (rc) return rc;
    double* cr = static_cast<double*>(chi);
    return ec_stage(E, cr, cr + mat, ec_dev, F_dev, true, chi0);
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
    std::vector<int> f(c->last_nw);
    HIP_TRY(hipMemcpy(f.data(), c->last_fail, sizeof(int) * c->last_nw, hipMemcpyDeviceToHost));
    for (int w = 0; w < c->last_nw; ++w)
        if (f[w])
            return fail(RPA_ERR_NOT_PD, "1 - K not positive definite at frequency index " + std::to_string(w) +
                                            " (pivot " + std::to_string(f[w] - 1) + ")");
    return RPA_OK;
}

}  // extern "C"
