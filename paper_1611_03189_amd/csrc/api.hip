// The extern "C" boundary (include/hsolve.h): argument checks, error translation,
// timing. No exception crosses it.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <new>

#include "hs_internal.h"

using hs::Error;
using hs::Plan;

struct hsolve_plan_s {
    Plan P;
    std::string last_error;
};

namespace {

hsolve_status guard(hsolve_plan plan, const char* where, void (*fn)(void*), void* arg) {
    try {
        fn(arg);
        return HSOLVE_OK;
    } catch (const Error& e) {
        if (plan) plan->last_error = std::string(where) + ": " + e.what;
        if (std::getenv("HSOLVE_VERBOSE")) std::fprintf(stderr, "hsolve %s: %s\n", where, e.what.c_str());
        return e.status;
    } catch (const std::bad_alloc&) {
        return HSOLVE_ERR_OOM;
    } catch (...) {
        return HSOLVE_ERR_DEVICE;
    }
}

struct ProfBind {             // make the plan's profiler visible to the launch wrappers
    explicit ProfBind(hsolve_plan plan) : prev(hs::t_prof) { hs::t_prof = plan ? &plan->P.prof : nullptr; }
    ~ProfBind() { hs::t_prof = prev; }
    hs::Profiler* prev;
};

template <class F>
hsolve_status run(hsolve_plan plan, const char* where, F&& f) {
    ProfBind bind(plan);
    return guard(plan, where, [](void* a) { (*static_cast<F*>(a))(); }, &f);
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

extern "C" {

void hsolve_default_options(hsolve_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->leaf_size = 16;
    o->eps = 1e-2;
    o->variant = HSOLVE_GC;
    o->nvec = 0;
    o->phi = nullptr;
    o->dim = 0;
    o->coords = nullptr;
    o->tol = 1e-10;
    o->max_iter = 1000;
    o->krylov = HSOLVE_PCG;
    o->stream = nullptr;
    o->apply_prec = 64;
    o->restart = 200;
    o->overlap_pivots = 1;
    o->factor_prec = 64;
    o->max_super = hs::MAX_SUPER;
    o->max_nrhs = 32;
    o->eps_schedule = HSOLVE_EPS_CONSTANT;
    o->cmp_lpe = 0;
    o->cmp_vectors = 0;
    o->apply_graph = 1;
    o->neighbours = HSOLVE_NEIGHBOURS_FOOTPRINT;
    o->eps1 = 0.0;
    o->cmp_ritz = 1;
    o->order = HSOLVE_ORDER_WAITING;
}

hsolve_status hsolve_analyze(int n, const int64_t* row_ptr, const int32_t* col_idx,
                             const hsolve_options* opt, hsolve_plan* out, size_t* arena_bytes_upper_bound) {
    if (!out) return HSOLVE_ERR_INVALID;
    *out = nullptr;
    if (arena_bytes_upper_bound) *arena_bytes_upper_bound = 0;
    if (n < 1 || !row_ptr || !col_idx) return HSOLVE_ERR_INVALID;
    hsolve_options o;
    if (opt) o = *opt;
    else hsolve_default_options(&o);
    if (!(o.eps >= 0.0) || !std::isfinite(o.eps) || o.leaf_size < 1 ||
        (o.variant != HSOLVE_LORASP && o.variant != HSOLVE_GC && o.variant != HSOLVE_GC_PROJ1) ||
        !(o.eps1 >= 0.0 && o.eps1 < 1.0) || o.dim < 0 || o.dim > 3 ||
        o.nvec < 0 || o.nvec > 8 || (o.phi && o.nvec < 1) || o.max_iter < 0 ||
        !(o.tol >= 0.0) || (o.krylov < HSOLVE_PCG || o.krylov > HSOLVE_STATIONARY) ||
        (o.apply_prec != 64 && o.apply_prec != 32) || o.restart < 1 ||
        (o.overlap_pivots != 0 && o.overlap_pivots != 1) || (o.factor_prec != 64 && o.factor_prec != 32) ||
        o.max_super < 1 || o.max_super > hs::MAX_SUPER || o.max_nrhs < 1 ||
        o.eps_schedule < HSOLVE_EPS_CONSTANT || o.eps_schedule > HSOLVE_EPS_GROW ||
        !(o.cmp_lpe == 0 || (o.cmp_lpe >= 1 && o.cmp_lpe <= 64 && (o.cmp_lpe & (o.cmp_lpe - 1)) == 0)) ||
        o.cmp_vectors < 0 || o.cmp_vectors > 2 || (o.apply_graph != 0 && o.apply_graph != 1) ||
        (o.cmp_ritz != 0 && o.cmp_ritz != 1) ||
        (o.order != HSOLVE_ORDER_INDEX && o.order != HSOLVE_ORDER_WAITING) ||
        (o.neighbours != HSOLVE_NEIGHBOURS_FOOTPRINT && o.neighbours != HSOLVE_NEIGHBOURS_GEOMETRIC))
        return HSOLVE_ERR_INVALID;
    if (row_ptr[0] != 0 || row_ptr[n] < 0) return HSOLVE_ERR_INVALID;
    hsolve_plan plan = new (std::nothrow) hsolve_plan_s();
    if (!plan) return HSOLVE_ERR_OOM;
    auto t0 = std::chrono::steady_clock::now();
    hsolve_status st = run(plan, "analyze", [&] {
        Plan& P = plan->P;
        P.n = n;
        P.nnz = row_ptr[n];
        P.opt = o;
        P.f32 = o.factor_prec == 32;
        P.apply32 = o.apply_prec == 32 || P.f32;      // an FP32 factor is applied in FP32
        if (P.f32) P.opt.apply_prec = 32;
        P.stream = static_cast<hipStream_t>(o.stream);
        P.row_ptr.assign(row_ptr, row_ptr + n + 1);
        P.col_idx.assign(col_idx, col_idx + P.nnz);
        if (o.coords && o.dim > 0) {
            P.coords.assign(o.coords, o.coords + size_t(n) * o.dim);
            for (double c : P.coords)
                if (!std::isfinite(c)) throw Error{HSOLVE_ERR_INVALID, "non-finite coordinate"};
        }
        P.opt.coords = P.coords.empty() ? nullptr : P.coords.data();
        if (o.variant == HSOLVE_GC || o.variant == HSOLVE_GC_PROJ1) {
            if (o.phi) {
                P.nphi = o.nvec;
                P.phi.assign(o.phi, o.phi + size_t(n) * o.nvec);
                for (double v : P.phi)
                    if (!std::isfinite(v)) throw Error{HSOLVE_ERR_INVALID, "non-finite phi"};
            } else {
                P.nphi = 1;
                P.phi.assign(size_t(n), 1.0);
            }
        }
        P.opt.phi = nullptr;
        hs::analyze(P);
        hs::size_arena(P);
        P.stats.arena_bound = int64_t(P.arena_bound);
        P.stats.levels = P.L;
        P.stats.colours = P.total_colours;
        P.stats.fail_level = P.stats.fail_node = -1;
    });
    if (st != HSOLVE_OK) {
        delete plan;
        return st;
    }
    plan->P.stats.t_analyze = seconds_since(t0);
    if (arena_bytes_upper_bound) *arena_bytes_upper_bound = plan->P.arena_bound;
    *out = plan;
    return HSOLVE_OK;
}

hsolve_status hsolve_factor(hsolve_plan plan, const double* values, void* d_arena, size_t arena_bytes) {
    if (!plan || !values || !d_arena) return HSOLVE_ERR_INVALID;
    Plan& P = plan->P;
    P.factored = false;
    return run(plan, "factor", [&] {
        hs::bind_arena(P, d_arena, arena_bytes);
        hs::factor(P, values);
    });
}

hsolve_status hsolve_apply(hsolve_plan plan, int nrhs, const double* r, int ldr, double* z,
                           int ldz) {
    if (!plan || !r || !z || nrhs < 1 || ldr < plan->P.n || ldz < plan->P.n)
        return HSOLVE_ERR_INVALID;
    if (!plan->P.factored) return HSOLVE_ERR_STATE;
    return run(plan, "apply", [&] {
        Plan& P = plan->P;
        hs::begin_workspace(P);
        const int batch = hs::solve_batch(P, nrhs, -1);
        for (int c0 = 0; c0 < nrhs; c0 += batch)
            hs::apply(P, std::min(batch, nrhs - c0), r + size_t(c0) * ldr, ldr, z + size_t(c0) * ldz, ldz);
        HS_HIP(hipStreamSynchronize(P.stream));
    });
}

hsolve_status hsolve_apply_static(hsolve_plan plan, int nrhs, const double* r, int ldr, double* z,
                                  int ldz) {
    if (!plan || !r || !z || nrhs < 1 || ldr < plan->P.n || ldz < plan->P.n)
        return HSOLVE_ERR_INVALID;
    if (!plan->P.factored) return HSOLVE_ERR_STATE;
    struct Args {
        hsolve_plan plan;
        int nrhs;
        const double* r;
        int ldr;
        double* z;
        int ldz;
    } args{plan, nrhs, r, ldr, z, ldz};
    // no kernel timing here: its events would be created on first use
    hs::Profiler* prev = hs::t_prof;
    hs::t_prof = nullptr;
    hsolve_status st = guard(plan, "apply_static", [](void* a) {
        const Args& q = *static_cast<const Args*>(a);
        hs::apply_static(q.plan->P, q.nrhs, q.r, q.ldr, q.z, q.ldz);
        HS_HIP(hipStreamSynchronize(q.plan->P.stream));
    }, &args);
    hs::t_prof = prev;
    return st;
}

hsolve_status hsolve_solve(hsolve_plan plan, int nrhs, const double* b, int ldb, double* x,
                           int ldx, hsolve_stats* stats) {
    if (!plan || !b || !x || nrhs < 1 || ldb < plan->P.n || ldx < plan->P.n)
        return HSOLVE_ERR_INVALID;
    Plan& P = plan->P;
    if (!P.factored) return HSOLVE_ERR_STATE;
    bool converged = true;
    auto t0 = std::chrono::steady_clock::now();
    hsolve_status st = run(plan, "solve", [&] {
        std::vector<int> its(nrhs);
        std::vector<double> rel(nrhs);
        hs::begin_workspace(P);
        const int batch = hs::solve_batch(P, nrhs, P.opt.krylov);
        for (int c0 = 0; c0 < nrhs; c0 += batch) {
            const int nc = std::min(batch, nrhs - c0);
            const double* bc = b + size_t(c0) * ldb;
            double* xc = x + size_t(c0) * ldx;
            if (P.opt.krylov == HSOLVE_STATIONARY)
                hs::stationary(P, nc, bc, ldb, xc, ldx, P.opt.tol, P.opt.max_iter, its.data() + c0, rel.data() + c0);
            else if (P.opt.krylov == HSOLVE_GMRES)
                hs::gmres(P, nc, bc, ldb, xc, ldx, P.opt.tol, P.opt.max_iter, P.opt.restart, its.data() + c0,
                          rel.data() + c0);
            else
                hs::pcg(P, nc, bc, ldb, xc, ldx, P.opt.tol, P.opt.max_iter, P.opt.krylov == HSOLVE_FPCG,
                        its.data() + c0, rel.data() + c0);
        }
        HS_HIP(hipStreamSynchronize(P.stream));
        int most = 0;
        double worst = 0.0;
        for (int c = 0; c < nrhs; ++c) {
            if (!(rel[c] <= P.opt.tol)) converged = false;
            most = std::max(most, its[c]);
            worst = std::max(worst, rel[c]);
        }
        P.stats.iterations = most;
        P.stats.rel_residual = worst;
    });
    P.stats.t_solve = seconds_since(t0);
    P.stats.device_bytes = int64_t(P.device_bytes());
    if (stats) *stats = P.stats;
    if (st != HSOLVE_OK) return st;
    return converged ? HSOLVE_OK : HSOLVE_NOT_CONVERGED;
}

hsolve_status hsolve_spmv(hsolve_plan plan, const double* x, double* y) {
    if (!plan || !x || !y) return HSOLVE_ERR_INVALID;
    if (!plan->P.factored) return HSOLVE_ERR_STATE;
    return run(plan, "spmv", [&] {
        hs::spmv(plan->P, x, y);
        HS_HIP(hipStreamSynchronize(plan->P.stream));
    });
}

size_t hsolve_tune_workspace_bytes(void) { return hs::tune_workspace_bytes(); }

hsolve_status hsolve_tune_gemm(void* d_work, size_t work_bytes, void* stream, int32_t* choice, double* ms) {
    if (!d_work) return HSOLVE_ERR_INVALID;
    return run(nullptr, "tune_gemm", [&] {
        std::vector<int> c(2 * hs::GEMM_BUCKETS, 0);
        hs::tune_gemm(d_work, work_bytes, static_cast<hipStream_t>(stream), c.data(), ms);
        if (choice)
            for (int b = 0; b < 2 * hs::GEMM_BUCKETS; ++b) choice[b] = c[b];
    });
}

hsolve_status hsolve_set_gemm_choice(const int32_t* choice) {
    if (!choice) return HSOLVE_ERR_INVALID;
    for (int b = 0; b < 2 * hs::GEMM_BUCKETS; ++b)
        if (choice[b] < 0 || choice[b] >= hs::GEMM_VARIANTS) return HSOLVE_ERR_INVALID;
    for (int b = 0; b < 2 * hs::GEMM_BUCKETS; ++b) hs::set_gemm_variant(b % hs::GEMM_BUCKETS, b >= hs::GEMM_BUCKETS, choice[b]);
    return HSOLVE_OK;
}

hsolve_status hsolve_set_stream(hsolve_plan plan, void* stream) {
    if (!plan) return HSOLVE_ERR_INVALID;
    plan->P.stream = static_cast<hipStream_t>(stream);
    plan->P.opt.stream = stream;
    return HSOLVE_OK;
}

hsolve_status hsolve_get_stats(hsolve_plan plan, hsolve_stats* stats) {
    if (!plan || !stats) return HSOLVE_ERR_INVALID;
    hs::Plan& P = plan->P;
    P.stats.device_bytes = int64_t(P.device_bytes());
    *stats = P.stats;
    return HSOLVE_OK;
}

hsolve_status hsolve_destroy(hsolve_plan plan) {
    if (!plan) return HSOLVE_OK;
    if (plan->P.arena) (void)hipStreamSynchronize(plan->P.stream);   // GPU used
    delete plan;
    return HSOLVE_OK;
}

const char* hsolve_status_string(hsolve_status s) {
    switch (s) {
        case HSOLVE_OK: return "HSOLVE_OK";
        case HSOLVE_NOT_CONVERGED: return "HSOLVE_NOT_CONVERGED";
        case HSOLVE_ERR_INVALID: return "HSOLVE_ERR_INVALID";
        case HSOLVE_ERR_NOT_SYMMETRIC: return "HSOLVE_ERR_NOT_SYMMETRIC";
        case HSOLVE_ERR_NOT_SPD: return "HSOLVE_ERR_NOT_SPD";
        case HSOLVE_ERR_OOM: return "HSOLVE_ERR_OOM";
        case HSOLVE_ERR_DEVICE: return "HSOLVE_ERR_DEVICE";
        case HSOLVE_ERR_STATE: return "HSOLVE_ERR_STATE";
        case HSOLVE_ERR_TOO_LARGE: return "HSOLVE_ERR_TOO_LARGE";
    }
    return "HSOLVE_UNKNOWN_STATUS";
}

hsolve_status hsolve_profile_begin(hsolve_plan plan) {
    if (!plan) return HSOLVE_ERR_INVALID;
    plan->P.prof.clear();
    plan->P.prof_totals.clear();
    plan->P.prof.on = true;
    return HSOLVE_OK;
}

hsolve_status hsolve_profile_only(hsolve_plan plan, const char* kernel) {
    if (!plan) return HSOLVE_ERR_INVALID;
    plan->P.prof.only = kernel ? kernel : "";
    return HSOLVE_OK;
}

hsolve_status hsolve_profile_end(hsolve_plan plan, int32_t* nkernels) {
    if (!plan) return HSOLVE_ERR_INVALID;
    plan->P.prof.on = false;
    hsolve_status st = run(plan, "profile_end", [&] { plan->P.prof_totals = plan->P.prof.totals(); });
    plan->P.prof.clear();
    if (nkernels) *nkernels = int32_t(plan->P.prof_totals.size());
    return st;
}

hsolve_status hsolve_profile_entry(hsolve_plan plan, int i, char* name, int cap, double* ms,
                                   int64_t* launches, double* work) {
    if (!plan || i < 0 || i >= int(plan->P.prof_totals.size())) return HSOLVE_ERR_INVALID;
    const hs::ProfTotal& t = plan->P.prof_totals[i];
    if (name && cap > 0) {
        std::strncpy(name, t.name.c_str(), size_t(cap) - 1);
        name[cap - 1] = 0;
    }
    if (ms) *ms = t.ms;
    if (launches) *launches = t.launches;
    if (work) *work = t.work;
    return HSOLVE_OK;
}

int hsolve_depth(hsolve_plan plan) { return plan ? plan->P.L : -1; }

const char* hsolve_last_error(hsolve_plan plan) {
    return plan ? plan->last_error.c_str() : "";
}

hsolve_status hsolve_leaf_order(hsolve_plan plan, int32_t* perm, int32_t* leaf_off) {
    if (!plan) return HSOLVE_ERR_INVALID;
    const Plan& P = plan->P;
    if (perm) std::memcpy(perm, P.perm.data(), sizeof(int32_t) * P.n);
    if (leaf_off) std::memcpy(leaf_off, P.leaf_off.data(), sizeof(int32_t) * P.leaf_off.size());
    return HSOLVE_OK;
}

hsolve_status hsolve_level_colours(hsolve_plan plan, int depth, int32_t* colour_of,
                                   int32_t* ncolours) {
    if (!plan || depth < 0 || depth >= int(plan->P.sym.size())) return HSOLVE_ERR_INVALID;
    const hs::LevelSym& S = plan->P.sym[depth];
    if (colour_of)
        for (size_t i = 0; i < S.colour_of.size(); ++i) colour_of[i] = S.colour_of[i];
    if (ncolours) *ncolours = int32_t(S.colours.size());
    return HSOLVE_OK;
}

hsolve_status hsolve_node_sets(hsolve_plan plan, int depth, int node, int32_t* nbrs, int32_t* nn,
                               int32_t* ws, int32_t* nw, int cap) {
    if (!plan || depth < 0 || depth >= int(plan->P.sym.size())) return HSOLVE_ERR_INVALID;
    const hs::LevelSym& S = plan->P.sym[depth];
    if (node < 0 || node >= int(S.N.size())) return HSOLVE_ERR_INVALID;
    if (nn) *nn = int32_t(S.N[node].size());
    if (nw) *nw = int32_t(S.W[node].size());
    for (size_t i = 0; nbrs && i < S.N[node].size() && int(i) < cap; ++i)
        nbrs[i] = 2 * S.N[node][i] + S.Nred[node][i];
    for (size_t i = 0; ws && i < S.W[node].size() && int(i) < cap; ++i)
        ws[i] = 2 * S.W[node][i] + S.Wred[node][i];
    return HSOLVE_OK;
}

hsolve_status hsolve_node_factor(hsolve_plan plan, int depth, int node, int32_t* dims,
                                 double* G, int64_t cap) {
    if (!plan || !dims || depth < 0 || depth >= int(plan->P.sym.size())) return HSOLVE_ERR_INVALID;
    const Plan& P = plan->P;
    if (!P.factored) return HSOLVE_ERR_STATE;
    const hs::LevelNum& LN = P.num[depth];
    if (node < 0 || node >= int(LN.node.size())) return HSOLVE_ERR_INVALID;
    const hs::NodeNum& nn = LN.node[node];
    dims[0] = nn.m;
    dims[1] = nn.ntot;
    dims[2] = nn.k;
    const int64_t count = int64_t(nn.ldG) * nn.m;
    if (!G || !nn.Gm || count == 0) return HSOLVE_OK;
    if (cap < count) return HSOLVE_ERR_INVALID;
    return run(plan, "node_factor", [&] {
        if (P.f32) {       // the FP32 factor, widened on the host
            std::vector<float> h(static_cast<size_t>(count));
            HS_HIP(hipMemcpy(h.data(), nn.Gm, sizeof(float) * count, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < count; ++i) G[i] = double(h[size_t(i)]);
        } else {
            HS_HIP(hipMemcpy(G, nn.Gm, sizeof(double) * count, hipMemcpyDeviceToHost));
        }
    });
}

hsolve_status hsolve_ranks(hsolve_plan plan, int depth, int32_t* ranks) {
    if (!plan || !ranks || depth < 0 || depth >= int(plan->P.sym.size())) return HSOLVE_ERR_INVALID;
    if (!plan->P.factored) return HSOLVE_ERR_STATE;
    const hs::LevelNum& LN = plan->P.num[depth];
    for (size_t i = 0; i < LN.ksz.size(); ++i) ranks[i] = LN.ksz[i];
    return HSOLVE_OK;
}

}  // extern "C"
