// Solve phase (Algorithm "Solve", §3.3) and the outer PCG.
//
// Solve-vector layout (one column): positions [0, n) hold the unknowns in leaf order;
// then, for depth d = L-1 .. 0, the red-node segments of that depth in index order.
// The super node s of depth d occupies the red segments of its two children (depth d+1),
// which are adjacent, so every node owns one contiguous segment.
//
// Per colour, in elimination order (forward) and in reverse (backward):
//   forward   phi_n -= T_n phi_s for every neighbour n, phi_r(s) = P_ss phi_s
//             (T_n = A_ns M_ss, so this is phi_n = r_n - A_ns M_ss r_s)
//   backward  x_s = M_ss phi_s - sum_n T_n^T x_n + P_ss^T x_r(s)
//             (= M_ss (b_s - A_sn x_n) + P_ss^T psi_r)
// The forward sweep updates V in place; the backward sweep reads phi from V and writes the
// solutions to a second vector X of the same layout, so the workgroups that share one node's
// columns never read a value that another of them has already replaced.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "hs_internal.h"

namespace hs {

// Four or more right-hand sides take the sweeps as grouped GEMMs on the matrix cores (a
// colour's targets, or its nodes, times the panel of right-hand sides), in 32 x 32 output
// tiles over at most APPLY_GEMM_COLS columns per launch: about 10 ms per 64^3 apply for 4 to
// 32 columns, against 11 and 33 ms for the row/column kernels, which stay for one to three
// columns (2.9 ms for one). Within either form a column's result does not depend on the
// other columns; the two forms differ by rounding.
constexpr int APPLY_GEMM_MIN_RHS = 4;
constexpr int APPLY_GEMM_VARIANT = 4;       // the 32 x 32 x 64 tile shape
constexpr int APPLY_GEMM_COLS = 32;

void build_apply_schedule(Plan& P) {
    const int L = P.L, nlev = std::max(L, 1);
    hipStream_t st = P.stream;
    // red segment offsets
    int64_t off = P.n;
    for (int d = nlev - 1; d >= 0; --d) {
        LevelNum& LN = P.num[d];
        LN.red_off.assign(size_t(1) << d, 0);
        for (int i = 0; i < (1 << d); ++i) {
            LN.red_off[i] = off;
            off += LN.ksz[i];
        }
    }
    P.vlen = off;
    auto super_off = [&](int d, int s) -> int64_t {
        if (L == 0) return 0;
        if (d == L - 1) return P.leaf_off[2 * s];
        return P.num[d + 1].red_off[2 * s];
    };
    // the factor copy the solve phase reads: Gm (double) or its single-precision copy
    const double w = P.apply32 ? 4.0 : 8.0;
    auto grow = [&](const NodeNum& nn, int row) -> const void* {
        if (P.apply32) return nn.Gm32 + row;
        return static_cast<const double*>(nn.Gm) + row;
    };
    double bytes = 0.0;
    P.sched.assign(nlev, {});
    // the tables of every colour land one after another in the factor region: their copies
    // merge into a few large ones, issued before the synchronisation below
    P.stage.begin_batch();
    for (int d = nlev - 1; d >= 0; --d) {
        const LevelSym& S = P.sym[d];
        const LevelNum& LN = P.num[d];
        P.sched[d].resize(S.colours.size());
        for (size_t c = 0; c < S.colours.size(); ++c) {
            std::map<int64_t, std::pair<FwdTarget, std::vector<FwdContrib>>> tg;
            std::vector<BwdNode> bn;
            std::vector<BwdSeg> bs;
            int max_rows = 0;
            for (int s : S.colours[c]) {
                const NodeNum& nn = LN.node[s];
                const int64_t src = super_off(d, s);
                for (size_t t = 0; t < S.N[s].size(); ++t) {
                    const int nb = S.N[s][t];
                    const bool red = S.Nred[s][t];
                    const int64_t dst = red ? LN.red_off[nb] : super_off(d, nb);
                    const int len = red ? LN.ksz[nb] : LN.msz[nb];
                    auto& e = tg[dst];
                    e.first = FwdTarget{dst, len, -1, 0, 0};
                    e.second.push_back(FwdContrib{grow(nn, nn.m + nn.noff[t]), src, nn.ldG, nn.m});
                }
                if (nn.k) {
                    const int64_t dst = LN.red_off[s];
                    auto& e = tg[dst];
                    e.first = FwdTarget{dst, nn.k, +1, 0, 0};
                    e.second.push_back(FwdContrib{grow(nn, nn.m + nn.ntot), src, nn.ldG, nn.m});
                }
                BwdNode b{grow(nn, 0), src, nn.ldG, nn.m, nn.m + nn.ntot + nn.k, int(bs.size()), 0, 0};
                bs.push_back(BwdSeg{src, nn.m, +1, 0, 0});
                for (size_t t = 0; t < S.N[s].size(); ++t) {
                    const int nb = S.N[s][t];
                    const bool red = S.Nred[s][t];
                    bs.push_back(BwdSeg{red ? LN.red_off[nb] : super_off(d, nb),
                                        red ? LN.ksz[nb] : LN.msz[nb], -1, 1, 0});
                }
                if (nn.k) bs.push_back(BwdSeg{LN.red_off[s], nn.k, +1, 1, 0});
                b.seg_end = int(bs.size());
                bn.push_back(b);
                max_rows = std::max(max_rows, b.rows);
                // factor reads: forward rows m.. of Gm, backward all rows; vectors twice
                bytes += w * (double(nn.ntot + nn.k) * nn.m + double(nn.ldG) * nn.m);
                bytes += w * 2.0 * (2.0 * nn.m + 2.0 * nn.ntot + 2.0 * nn.k);
            }
            std::vector<FwdTarget> ft;
            std::vector<FwdContrib> fc;
            int max_len = 0;
            for (auto& [dst, e] : tg) {
                FwdTarget t = e.first;
                t.c_begin = int(fc.size());
                fc.insert(fc.end(), e.second.begin(), e.second.end());
                t.c_end = int(fc.size());
                ft.push_back(t);
                max_len = std::max(max_len, t.len);
            }
            Plan::ColourSched& cs = P.sched[d][c];
            for (int s : S.colours[c]) {
                const NodeNum& nn = LN.node[s];
                cs.fwd_bytes += w * (double(nn.ntot + nn.k) * nn.m + nn.m + 2.0 * (nn.ntot + nn.k));
                cs.bwd_bytes += w * (double(nn.ldG) * nn.m + nn.ldG + nn.m);
            }
            // the GEMM forms: offsets into V (base 0) and X (base 1), N set by the launch
            const GemmShape& gsh = GEMM_SHAPES[APPLY_GEMM_VARIANT];
            const int ldvi = int(P.vlen);
            auto rel = [](int64_t off) { return reinterpret_cast<void*>(uintptr_t(off)); };
            auto upload_gemm = [&](std::vector<GemmTask>& tk, std::vector<GemmTerm>& tm, Plan::ApplyGemm& ag) {
                std::vector<GemmTile> tl;
                for (size_t id = 0; id < tk.size(); ++id)
                    for (int ti = 0; ti * gsh.tm < tk[id].M; ++ti) tl.push_back(GemmTile{int(id), ti, 0, 0});
                ag.ntiles = int(tl.size());
                if (tl.empty()) return;
                ag.tasks = P.stage.upload_vec(tk, P.fpool, st);
                ag.terms = P.stage.upload_vec(tm, P.fpool, st);
                ag.tiles = P.stage.upload_vec(tl, P.fpool, st);
            };
            {
                std::vector<GemmTask> tk;
                std::vector<GemmTerm> tm;
                for (const FwdTarget& t : ft) {
                    if (t.len <= 0) continue;
                    GemmTask g{rel(t.dst), ldvi, t.len, 0, int(tm.size()), int(tm.size()), GEMM_REL, double(t.sign), 1.0};
                    for (int q = t.c_begin; q < t.c_end; ++q) {
                        const FwdContrib& f = fc[q];
                        if (f.m <= 0) continue;
                        tm.push_back(GemmTerm{f.G, rel(f.src), f.ldG, ldvi, f.m, 0, 0, GEMM_REL});
                        cs.gf.flops += 2.0 * t.len * f.m;
                    }
                    g.t_end = int(tm.size());
                    tk.push_back(g);
                }
                upload_gemm(tk, tm, cs.gf);
            }
            {
                std::vector<GemmTask> tk;
                std::vector<GemmTerm> tm;
                for (const BwdNode& b : bn) {
                    if (b.m <= 0) continue;
                    GemmTask g{rel(b.dst), ldvi, b.m, 0, int(tm.size()), int(tm.size()), GEMM_REL | GEMM_BASE1, 1.0, 0.0};
                    int pos = 0;
                    for (int q = b.seg_begin; q < b.seg_end; ++q) {
                        const BwdSeg& sg = bs[q];
                        if (sg.len > 0) {
                            const void* A = static_cast<const char*>(b.G) + size_t(pos) * (P.apply32 ? 4 : 8);
                            const int fl = GEMM_REL | (sg.buf ? GEMM_BASE1 : 0) | (sg.sign < 0 ? GEMM_NEG : 0);
                            tm.push_back(GemmTerm{A, rel(sg.off), b.ldG, ldvi, sg.len, 1, 0, fl});
                            cs.gb.flops += 2.0 * b.m * sg.len;
                        }
                        pos += sg.len;
                    }
                    g.t_end = int(tm.size());
                    tk.push_back(g);
                }
                upload_gemm(tk, tm, cs.gb);
            }
            cs.nfwd = int(ft.size());
            cs.max_len = max_len;
            cs.fwd_t = P.stage.upload_vec(ft, P.fpool, st);
            cs.fwd_c = P.stage.upload_vec(fc, P.fpool, st);
            cs.nbwd = int(bn.size());
            for (const BwdNode& b : bn) cs.max_m = std::max(cs.max_m, b.m);
            cs.bwd_n = P.stage.upload_vec(bn, P.fpool, st);
            cs.bwd_s = P.stage.upload_vec(bs, P.fpool, st);
            if (max_rows > 6144 && !P.dry)
                throw Error{HSOLVE_ERR_INVALID, "super node with too many neighbour rows for the solve kernel"};
        }
    }
    P.stats.apply_bytes = bytes + (8.0 + w) * P.n;
    P.stage.end_batch(st);
    if (!P.dry) HS_HIP(hipStreamSynchronize(st));
    P.stage.reset();
}

// The solve phase of one API call takes its vectors from the arena above the factor data
// (the transient regions of the factorization are free by then); calls on a plan do not
// overlap, so each call starts the workspace afresh.
void begin_workspace(Plan& P) {
    char* end = P.arena + P.arena_bytes;
    P.wpool.init(P.fpool.top(), size_t(end - P.fpool.top()), "solve workspace");
    P.d_V = P.d_X = nullptr;
    P.V_cols = 0;
    P.d_krylov = nullptr;
    P.krylov_cols = 0;
    P.d_gmres = nullptr;
    P.gmres_restart = 0;
}

static void ensure_V(Plan& P, int nrhs) {
    if (P.d_V && P.V_cols >= nrhs) return;
    const size_t bytes = (P.apply32 ? sizeof(float) : sizeof(double)) * size_t(P.vlen) * nrhs;
    P.d_V = P.wpool.alloc(bytes);
    P.d_X = P.wpool.alloc(bytes);
    P.V_cols = nrhs;
}

// The sweeps of one apply on V / X: zero the red segments, forward colour by colour from the
// leaves up, backward from the root down.
template <typename T>
static void sweeps(Plan& P, int nrhs, T* V, T* X, hipStream_t st) {
    const int L = P.L, nlev = std::max(L, 1);
    const int64_t ldv = P.vlen;
    for (int c = 0; c < nrhs; ++c) launch_fill<T>(V + size_t(c) * ldv + P.n, T(0), P.vlen - P.n, st);
    if (nrhs >= APPLY_GEMM_MIN_RHS) {
        auto run = [&](const Plan::ApplyGemm& ag, const char* name) {
            for (int c0 = 0; c0 < nrhs; c0 += APPLY_GEMM_COLS) {
                const int nc = std::min(APPLY_GEMM_COLS, nrhs - c0);
                launch_gemm<T>(ag.tasks, ag.terms, ag.tiles, ag.ntiles, ag.flops * nc, APPLY_GEMM_VARIANT, st,
                               V + size_t(c0) * ldv, X + size_t(c0) * ldv, nc, name);
            }
        };
        for (int d = nlev - 1; d >= 0; --d)
            for (size_t c = 0; c < P.sched[d].size(); ++c) run(P.sched[d][c].gf, "k_fwd_gemm");
        for (int d = 0; d < nlev; ++d)
            for (size_t c = P.sched[d].size(); c-- > 0;) run(P.sched[d][c].gb, "k_bwd_gemm");
        return;
    }
    for (int d = nlev - 1; d >= 0; --d)
        for (size_t c = 0; c < P.sched[d].size(); ++c) {
            const Plan::ColourSched& cs = P.sched[d][c];
            launch_fwd<T>(cs.fwd_t, cs.fwd_c, cs.nfwd, cs.max_len, V, ldv, nrhs, cs.fwd_bytes * nrhs, st);
        }
    for (int d = 0; d < nlev; ++d)
        for (size_t c = P.sched[d].size(); c-- > 0;) {
            const Plan::ColourSched& cs = P.sched[d][c];
            launch_bwd<T>(cs.bwd_n, cs.bwd_s, cs.nbwd, cs.max_m, V, X, ldv, nrhs, cs.bwd_bytes * nrhs, st);
        }
}

// The sweeps as one HIP graph, captured on the plan's capture stream the first time a
// (V, X, nrhs) triple is seen after a factorization and replayed on the plan's stream after
// that: the 2 x (colours) dependent launches of an apply are submitted as one. The graph
// holds kernel nodes only (the red segments are zeroed by a fill kernel, not a memset).
template <typename T>
static hipGraphExec_t sweep_graph(Plan& P, int nrhs, T* V, T* X) {
    for (const Plan::Graph& g : P.graphs)
        if (g.V == V && g.X == X && g.nrhs == nrhs) return g.exec;
    if (!P.cap) HS_HIP(hipStreamCreateWithFlags(&P.cap, hipStreamNonBlocking));
    if (P.graphs.size() >= 8) {      // a few workspaces at most; drop the oldest
        (void)hipGraphExecDestroy(P.graphs.front().exec);
        P.graphs.erase(P.graphs.begin());
    }
    hipGraph_t graph = nullptr;
    HS_HIP(hipStreamBeginCapture(P.cap, hipStreamCaptureModeThreadLocal));
    try {
        sweeps<T>(P, nrhs, V, X, P.cap);
    } catch (...) {
        (void)hipStreamEndCapture(P.cap, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HS_HIP(hipStreamEndCapture(P.cap, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) throw Error{HSOLVE_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    P.graphs.push_back(Plan::Graph{V, X, nrhs, exec});
    return exec;
}

template <typename T>
static void apply_t(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz, bool graph) {
    hipStream_t st = P.stream;
    const int64_t ldv = P.vlen;
    T* V = static_cast<T*>(P.d_V);
    T* X = static_cast<T*>(P.d_X);
    launch_gather_perm<T>(r, ldr, V, ldv, P.d_perm, P.n, nrhs, st);
    // kernel timing records every launch: it takes the eager path
    if (graph && P.opt.apply_graph && !(t_prof && t_prof->on)) HS_HIP(hipGraphLaunch(sweep_graph<T>(P, nrhs, V, X), st));
    else sweeps<T>(P, nrhs, V, X, st);
    launch_scatter_perm<T>(X, ldv, z, ldz, P.d_perm, P.n, nrhs, st);
}

void clear_graphs(Plan& P) {
    for (Plan::Graph& g : P.graphs) (void)hipGraphExecDestroy(g.exec);
    P.graphs.clear();
}

// z = A_H^{-1} r for nrhs columns (device pointers, original unknown order); the sweeps run in
// the precision of the factor copy the plan keeps for them
void apply(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz, bool graph) {
    if (!P.factored) throw Error{HSOLVE_ERR_STATE, "apply before factor"};
    ensure_V(P, nrhs);
    if (P.apply32) apply_t<float>(P, nrhs, r, ldr, z, ldz, graph);
    else apply_t<double>(P, nrhs, r, ldr, z, ldz, graph);
}

// ---------------------------------------------------------------------------------
// Apply with the solve vectors in the library's static device scratch (hsolve_apply_static):
// for callers that cannot allocate. `scratch` is a file-scope device array; host code uses
// only the address hipGetSymbolAddress returns for the current device (the array's name is
// a host-side stand-in, not a device address). Every plan on a GPU shares that GPU's copy.
// ---------------------------------------------------------------------------------
static __device__ __align__(256) char scratch[APPLY_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static void* scratch_on_current_device() {
    int dev = 0;
    HS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) throw Error{HSOLVE_ERR_DEVICE, "device index out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{HSOLVE_ERR_DEVICE, "no device address for the static scratch"};
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// z = A_H^{-1} r with V and X in the static scratch: the same kernels and schedule as apply(),
// no workspace from the arena and no allocation. The red segments of V are cleared by the
// apply itself, so the scratch's previous contents do not matter.
void apply_static(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz) {
    if (!P.factored) throw Error{HSOLVE_ERR_STATE, "apply before factor"};
    const size_t w = P.apply32 ? sizeof(float) : sizeof(double);
    const size_t half = align256(w * size_t(P.vlen) * nrhs);
    if (2 * half > APPLY_SCRATCH_BYTES)
        throw Error{HSOLVE_ERR_OOM, "the solve vectors need " + std::to_string(2 * half) +
                                        " bytes; the static scratch holds " + std::to_string(APPLY_SCRATCH_BYTES)};
    char* base = static_cast<char*>(scratch_on_current_device());
    P.d_V = base;
    P.d_X = base + half;
    P.V_cols = nrhs;
    apply(P, nrhs, r, ldr, z, ldz, /*graph=*/false);     // instantiating a graph would allocate
    // later calls on the plan must not take these pointers for their arena workspace
    P.d_V = P.d_X = nullptr;
    P.V_cols = 0;
}

void spmv(Plan& P, const double* x, double* y) {
    launch_spmv(P.d_row_ptr, P.d_col_idx, P.d_values, x, y, P.n, P.nnz, P.stream);
}

// PCG (Hestenes-Stiefel) with x0 = 0 on nrhs columns at once, each with its own scalars: a
// column stops changing once ||r_k|| <= tol ||b|| (by the recursion). One SpMV, one apply and
// one scalar read-back per iteration for the whole block. its[c] and rel[c] receive the
// iteration count and the final recursive relative residual of column c.
// flexible: beta_k = r_{k+1}^T (z_{k+1} - z_k) / r_k^T z_k (Polak-Ribiere form), which keeps the
// iteration convergent when the preconditioner is applied in lower precision; r_{k+1}^T z_k is
// taken before the apply overwrites z_k. With an exact symmetric preconditioner it equals the
// standard beta in exact arithmetic.
void pcg(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
         bool flexible, int* its, double* rel) {
    hipStream_t st = P.stream;
    const int n = P.n;
    const int64_t ld = n;
    if (!P.d_krylov || P.krylov_cols < nrhs) {
        P.d_krylov = P.wpool.alloc_n<double>(size_t(n) * 5 * nrhs);
        P.d_kscal = P.wpool.alloc_n<double>(size_t(nrhs) * (6 + DOTM_BLOCKS));
        P.d_kflag = P.wpool.alloc_n<int>(size_t(nrhs));
        P.krylov_cols = nrhs;
    }
    if (!P.h_scalars || P.h_scalar_cols < nrhs) {
        if (P.h_scalars) HS_HIP(hipHostFree(P.h_scalars));
        HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_scalars), sizeof(double) * 3 * size_t(nrhs) + 64,
                             hipHostMallocDefault));
        P.h_scalar_cols = nrhs;
    }
    double* R = P.d_krylov;
    double* Z = R + size_t(n) * nrhs;
    double* Pv = Z + size_t(n) * nrhs;
    double* Q = Pv + size_t(n) * nrhs;
    double* X = Q + size_t(n) * nrhs;
    double* bb = P.d_kscal;                     // ||b||^2, then ||b||
    double* rz = bb + nrhs;
    double* pq = rz + nrhs;
    double* rr = pq + nrhs;
    double* rzn = rr + nrhs;
    double* rzo = rzn + nrhs;                   // flexible: r_{k+1}^T z_k
    double* part = rzn + 2 * nrhs;              // DOTM_BLOCKS partial sums per column
    int* active = P.d_kflag;
    double* h = P.h_scalars;                    // host: ||b||, rr, active (as doubles)
    int* hact = reinterpret_cast<int*>(h + 2 * size_t(nrhs));
    HS_HIP(hipMemcpy2DAsync(R, sizeof(double) * ld, b, sizeof(double) * size_t(ldb), sizeof(double) * n, nrhs,
                            hipMemcpyDeviceToDevice, st));
    launch_fill(X, 0.0, int64_t(n) * nrhs, st);
    auto copy_out = [&] {
        HS_HIP(hipMemcpy2DAsync(x, sizeof(double) * size_t(ldx), X, sizeof(double) * ld, sizeof(double) * n, nrhs,
                                hipMemcpyDeviceToDevice, st));
    };
    launch_dots(R, R, ld, n, nrhs, part, bb, st);
    HS_HIP(hipMemcpyAsync(h, bb, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HS_HIP(hipStreamSynchronize(st));
    bool any = false;
    for (int c = 0; c < nrhs; ++c)
        if (!std::isfinite(h[c])) throw Error{HSOLVE_ERR_INVALID, "right-hand side contains NaN or Inf"};
    for (int c = 0; c < nrhs; ++c) {
        h[c] = std::sqrt(h[c]);
        hact[c] = h[c] > 0.0 ? 1 : 0;
        any = any || hact[c];
        its[c] = 0;
        rel[c] = 0.0;
    }
    HS_HIP(hipMemcpyAsync(bb, h, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    HS_HIP(hipMemcpyAsync(active, hact, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    HS_HIP(hipStreamSynchronize(st));            // the host buffer is reused below
    if (!any) {
        copy_out();
        return;
    }
    std::vector<double> nbh(h, h + nrhs);
    std::vector<int> live(hact, hact + nrhs);
    apply(P, nrhs, R, n, Z, n);
    HS_HIP(hipMemcpyAsync(Pv, Z, sizeof(double) * size_t(n) * nrhs, hipMemcpyDeviceToDevice, st));
    launch_dots(R, Z, ld, n, nrhs, part, rz, st);
    int it = 0;
    while (it < max_iter) {
        launch_spmv_multi(P.d_row_ptr, P.d_col_idx, P.d_values, Pv, ld, Q, ld, n, nrhs, P.nnz, st);
        launch_dots(Pv, Q, ld, n, nrhs, part, pq, st);
        launch_axpy2_multi(X, Pv, R, Q, ld, n, nrhs, rz, pq, active, st);
        ++it;
        launch_dots(R, R, ld, n, nrhs, part, rr, st);
        launch_pcg_flags(rr, bb, tol, active, nullptr, nullptr, nrhs, st);
        HS_HIP(hipMemcpyAsync(h + nrhs, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
        HS_HIP(hipMemcpyAsync(hact, active, sizeof(int) * nrhs, hipMemcpyDeviceToHost, st));
        HS_HIP(hipStreamSynchronize(st));
        any = false;
        for (int c = 0; c < nrhs; ++c) {
            if (!live[c]) continue;
            its[c] = it;
            rel[c] = std::sqrt(h[nrhs + c]) / nbh[c];
            if (!hact[c]) live[c] = 0;
            any = any || live[c];
        }
        if (!any) break;
        if (flexible) launch_dots(R, Z, ld, n, nrhs, part, rzo, st);
        apply(P, nrhs, R, n, Z, n);
        launch_dots(R, Z, ld, n, nrhs, part, rzn, st);
        launch_xpby_multi(Pv, Z, ld, n, nrhs, rzn, flexible ? rzo : nullptr, rz, active, st);
        launch_copy_scalars(rz, rzn, nrhs, st);
    }
    copy_out();
}

// Stationary iteration x_{k+1} = x_k + A_H^{-1}(b - A x_k), x_0 = 0 (§7.1), all columns
// together: one apply, one SpMV and one read-back of the residual norms per iteration. A
// column stops changing once ||b - A x_k|| <= tol ||b|| (the residual is the true one).
void stationary(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
                int* its, double* rel) {
    hipStream_t st = P.stream;
    const int n = P.n;
    const int64_t ld = n;
    if (!P.d_krylov || P.krylov_cols < nrhs) {
        P.d_krylov = P.wpool.alloc_n<double>(size_t(n) * 5 * nrhs);
        P.d_kscal = P.wpool.alloc_n<double>(size_t(nrhs) * (6 + DOTM_BLOCKS));
        P.d_kflag = P.wpool.alloc_n<int>(size_t(nrhs));
        P.krylov_cols = nrhs;
    }
    if (!P.h_scalars || P.h_scalar_cols < nrhs) {
        if (P.h_scalars) HS_HIP(hipHostFree(P.h_scalars));
        HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_scalars), sizeof(double) * 3 * size_t(nrhs) + 64,
                             hipHostMallocDefault));
        P.h_scalar_cols = nrhs;
    }
    double* R = P.d_krylov;
    double* Z = R + size_t(n) * nrhs;
    double* Q = Z + size_t(n) * nrhs;
    double* X = Q + size_t(n) * nrhs;
    double* rr = P.d_kscal;
    double* part = rr + 6 * size_t(nrhs);
    int* active = P.d_kflag;
    double* h = P.h_scalars;
    int* hact = reinterpret_cast<int*>(h + 2 * size_t(nrhs));
    HS_HIP(hipMemcpy2DAsync(R, sizeof(double) * ld, b, sizeof(double) * size_t(ldb), sizeof(double) * n, nrhs,
                            hipMemcpyDeviceToDevice, st));
    launch_fill<double>(X, 0.0, int64_t(n) * nrhs, st);
    launch_dots(R, R, ld, n, nrhs, part, rr, st);
    HS_HIP(hipMemcpyAsync(h, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HS_HIP(hipStreamSynchronize(st));
    std::vector<double> nb(nrhs);
    bool any = false;
    for (int c = 0; c < nrhs; ++c)
        if (!std::isfinite(h[c])) throw Error{HSOLVE_ERR_INVALID, "right-hand side contains NaN or Inf"};
    for (int c = 0; c < nrhs; ++c) {
        nb[c] = std::sqrt(h[c]);
        hact[c] = nb[c] > 0.0 ? 1 : 0;
        any = any || hact[c];
        its[c] = 0;
        rel[c] = 0.0;
    }
    HS_HIP(hipMemcpyAsync(active, hact, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
    HS_HIP(hipStreamSynchronize(st));
    std::vector<int> live(hact, hact + nrhs);
    for (int it = 1; any && it <= max_iter; ++it) {
        apply(P, nrhs, R, n, Z, n);
        launch_add_multi(X, Z, ld, n, nrhs, active, st);
        launch_spmv_multi(P.d_row_ptr, P.d_col_idx, P.d_values, X, ld, Q, ld, n, nrhs, P.nnz, st);
        launch_sub_multi(R, b, ldb, Q, ld, n, nrhs, active, st);
        launch_dots(R, R, ld, n, nrhs, part, rr, st);
        HS_HIP(hipMemcpyAsync(h, rr, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
        HS_HIP(hipStreamSynchronize(st));
        any = false;
        for (int c = 0; c < nrhs; ++c) {
            if (!live[c]) continue;
            its[c] = it;
            rel[c] = std::sqrt(h[c]) / nb[c];
            if (!(rel[c] > tol)) live[c] = 0;
            hact[c] = live[c];
            any = any || live[c];
        }
        HS_HIP(hipMemcpyAsync(active, hact, sizeof(int) * nrhs, hipMemcpyHostToDevice, st));
        HS_HIP(hipStreamSynchronize(st));        // the host flags are rewritten next iteration
    }
    HS_HIP(hipMemcpy2DAsync(x, sizeof(double) * size_t(ldx), X, sizeof(double) * ld, sizeof(double) * n, nrhs,
                            hipMemcpyDeviceToDevice, st));
}

// Restarted GMRES, right-preconditioned (A M y = b, x = M y), one column at a time, x0 = 0:
// Arnoldi with modified Gram-Schmidt (coefficients stay on the device), the preconditioned
// basis Z kept so that x += Z y also holds when M varies slightly between calls (single-
// precision solve phase); Givens rotations and the small triangular solve on the host, one
// read-back of the new Hessenberg column per step. Stops when the residual estimate |g_{j+1}|
// reaches tol ||b|| (the true residual for right preconditioning, up to rounding); rel[c] is
// the true relative residual recomputed at the end.
void gmres(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
           int restart, int* its, double* rel) {
    hipStream_t st = P.stream;
    const int n = P.n;
    const int m = std::max(1, restart);
    if (!P.d_gmres || P.gmres_restart < m) {
        P.d_gmres = P.wpool.alloc_n<double>(size_t(n) * (2 * size_t(m) + 4) + size_t(m + 2) + DOTM_BLOCKS + 8);
        P.gmres_restart = m;
    }
    if (!P.h_scalars || P.h_scalar_cols < m + 8) {
        if (P.h_scalars) HS_HIP(hipHostFree(P.h_scalars));
        HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_scalars), sizeof(double) * 3 * size_t(m + 8) + 64,
                             hipHostMallocDefault));
        P.h_scalar_cols = m + 8;
    }
    double* Vb = P.d_gmres;                          // n x (m + 1)
    double* Zb = Vb + size_t(n) * (m + 1);           // n x m
    double* w = Zb + size_t(n) * m;
    double* r = w + n;
    double* X = r + n;
    double* hcol = X + n;                            // m + 2 Hessenberg entries of one column
    double* part = hcol + (m + 2);
    double* h = P.h_scalars;
    auto dot = [&](const double* a, const double* bb, double* out) { launch_dots(a, bb, n, n, 1, part, out, st); };
    auto read = [&](const double* src, int cnt) {
        HS_HIP(hipMemcpyAsync(h, src, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
        HS_HIP(hipStreamSynchronize(st));
    };
    std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    for (int c = 0; c < nrhs; ++c) {
        const double* bc = b + size_t(c) * ldb;
        launch_fill<double>(X, 0.0, n, st);
        dot(bc, bc, hcol);
        read(hcol, 1);
        if (!std::isfinite(h[0])) throw Error{HSOLVE_ERR_INVALID, "right-hand side contains NaN or Inf"};
        const double nb = std::sqrt(h[0]);
        int total = 0;
        while (nb > 0.0 && total < max_iter) {
            launch_spmv(P.d_row_ptr, P.d_col_idx, P.d_values, X, w, n, P.nnz, st);
            launch_sub(r, bc, w, n, st);
            dot(r, r, hcol);
            read(hcol, 1);
            const double beta = std::sqrt(h[0]);
            if (beta / nb <= tol) break;
            const int mm = std::min(m, max_iter - total);
            std::fill(H.begin(), H.end(), 0.0);
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            launch_scale(Vb, r, 1.0 / beta, n, st);
            int jd = 0;
            for (int j = 0; j < mm; ++j) {
                double* vj = Vb + size_t(n) * j;
                double* zj = Zb + size_t(n) * j;
                apply(P, 1, vj, n, zj, n);
                launch_spmv(P.d_row_ptr, P.d_col_idx, P.d_values, zj, w, n, P.nnz, st);
                for (int i = 0; i <= j; ++i) {
                    dot(w, Vb + size_t(n) * i, hcol + i);
                    launch_axpy_dev(w, Vb + size_t(n) * i, hcol + i, -1.0, n, st);
                }
                dot(w, w, hcol + j + 1);
                read(hcol, j + 2);
                double* Hj = H.data() + size_t(j) * (m + 1);   // column j, m + 1 rows
                for (int i = 0; i <= j; ++i) Hj[i] = h[i];
                Hj[j + 1] = std::sqrt(h[j + 1]);
                if (Hj[j + 1] > 0.0) launch_scale(Vb + size_t(n) * (j + 1), w, 1.0 / Hj[j + 1], n, st);
                for (int i = 0; i < j; ++i) {
                    const double t = cs[i] * Hj[i] + sn[i] * Hj[i + 1];
                    Hj[i + 1] = -sn[i] * Hj[i] + cs[i] * Hj[i + 1];
                    Hj[i] = t;
                }
                const double den = std::hypot(Hj[j], Hj[j + 1]);
                cs[j] = Hj[j] / den;
                sn[j] = Hj[j + 1] / den;
                Hj[j] = den;
                Hj[j + 1] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++total;
                jd = j + 1;
                if (std::fabs(g[j + 1]) / nb <= tol) break;
            }
            for (int i = jd - 1; i >= 0; --i) {      // back substitution with the triangle of H
                double t = g[i];
                for (int k = i + 1; k < jd; ++k) t -= H[size_t(k) * (m + 1) + i] * y[k];
                y[i] = t / H[size_t(i) * (m + 1) + i];
            }
            std::memcpy(h, y.data(), sizeof(double) * jd);
            HS_HIP(hipMemcpyAsync(hcol, h, sizeof(double) * jd, hipMemcpyHostToDevice, st));
            launch_gemv_acc(X, Zb, n, hcol, jd, n, st);
            HS_HIP(hipStreamSynchronize(st));        // h is reused as a read-back buffer
            if (std::fabs(g[jd]) / nb <= tol) break;
        }
        // true residual
        launch_spmv(P.d_row_ptr, P.d_col_idx, P.d_values, X, w, n, P.nnz, st);
        launch_sub(r, bc, w, n, st);
        dot(r, r, hcol);
        read(hcol, 1);
        its[c] = total;
        rel[c] = nb > 0.0 ? std::sqrt(h[0]) / nb : 0.0;
        HS_HIP(hipMemcpyAsync(x + size_t(c) * ldx, X, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    HS_HIP(hipStreamSynchronize(st));
}

}  // namespace hs
