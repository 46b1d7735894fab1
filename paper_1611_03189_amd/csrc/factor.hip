// Numeric factorization (Algorithm "Setup"), driven level by level and colour by colour.
//
// For every colour of a level all its super nodes are processed together (they share no
// block, so this equals eliminating them one after the other, §3.2 "a given ordering"):
//   A  compression (§3.2 eq. local_compression; §6 eq. compression_xy / preserve):
//      gather A_sw, Gram matrix, [phi_s, A_sw phi_w] for GC, eigen-decomposition and
//      truncation on the GPU; the ranks k come back to the host (they size the new blocks)
//   B  elimination (§3.2 eq. extended_rearranged, K = L K2 L^T; Appendix A):
//      A_ss^-1, Y = A_ss^-1 U, S = U^T Y, S^-1, P_ss = S^-1 Y^T, M_ss = A_ss^-1 - Y P_ss,
//      T_N = A_Ns M_ss (kept for the solve), red-node blocks S^-1, A_ns P_ss^T, R,
//      the preserved vector U^T phi_s, and the Schur update A_n1n2 -= T_n1 A_n2s^T
//      (gathered per target block, contributions in index order).
// At the end of a level the red nodes of sibling pairs are merged into the super nodes
// of the parent level (Algorithm "Setup", merge step).
#include <algorithm>
#include <cstring>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "hs_internal.h"

namespace hs {

namespace {

struct Live {
    std::unordered_map<uint64_t, Block> map;
    Block* find(int i, int j) {
        auto it = map.find(i <= j ? bkey(i, j) : bkey(j, i));
        return it == map.end() ? nullptr : &it->second;
    }
    void put(int i, int j, const Block& b) { map[bkey(i, j)] = b; }   // i <= j
    void erase(int i, int j) { map.erase(i <= j ? bkey(i, j) : bkey(j, i)); }
};

template <typename R>
struct Batch {
    bool trace_pivots = false;
    bool dry = false;                 // replay: tables are counted, nothing is launched
    std::vector<CopyTask> copies;
    std::vector<GemmTask> gt;
    std::vector<GemmTerm> terms;
    std::vector<GemmTile> tiles;
    std::vector<CholTask> chol;

    void copy(const R* src, int lds, R* dst, int ldd, int rows, int cols, int trans) {
        if (rows > 0 && cols > 0) copies.push_back(CopyTask{src, dst, lds, ldd, rows, cols, trans, 0});
    }
    void open(R* C, int ldc, int M, int N, double alpha, double beta) {
        gt.push_back(GemmTask{C, ldc, M, N, int(terms.size()), int(terms.size()), 0, alpha, beta});
    }
    void term(const R* A, int lda, int tA, const R* B, int ldb, int tB, int K) {
        if (K <= 0) return;
        terms.push_back(GemmTerm{A, B, lda, ldb, K, tA, tB, 0});
        gt.back().t_end = int(terms.size());
    }
    void close() {}   // output tiles are laid out at flush time, in the launch's tile shape
    void gemm(R* C, int ldc, int M, int N, double alpha, double beta, const R* A,
              int lda, int tA, const R* B, int ldb, int tB, int K) {
        if (M <= 0 || N <= 0) return;
        open(C, ldc, M, N, alpha, beta);
        term(A, lda, tA, B, ldb, tB, K);
        close();
    }
    // C (M x M) = alpha A op(A) for a symmetric result: only the tiles on or below the
    // diagonal are computed, and their lower values are mirrored (GEMM_MIRROR)
    void gemm_sym(R* C, int ldc, int M, double alpha, const R* A, int lda, int tA, int K) {
        if (M <= 0) return;
        open(C, ldc, M, M, alpha, 0.0);
        gt.back().flags |= GEMM_MIRROR;
        term(A, lda, tA, A, lda, 1 - tA, K);
        close();
    }
    void flush_copies(Plan& P) {
        if (copies.empty()) return;
        double bytes = 0.0;
        int max_cols = 0;
        for (const CopyTask& c : copies) {
            bytes += 2.0 * sizeof(R) * c.rows * c.cols;
            max_cols = std::max(max_cols, c.cols);
        }
        CopyTask* d = P.stage.upload_vec(copies, P.spool, P.stream);
        if (!dry) launch_copy<R>(d, int(copies.size()), max_cols, bytes, P.stream);
        copies.clear();
    }
    // The tables always travel on the plan's stream; with side set, the launch goes to the
    // side stream once it has waited for them.
    static hipStream_t to_side(Plan& P, bool side) {
        if (!side || P.dry) return P.stream;
        HS_HIP(hipEventRecord(P.ev_ready, P.stream));
        HS_HIP(hipStreamWaitEvent(P.side, P.ev_ready, 0));
        return P.side;
    }
    void flush_gemm(Plan& P, bool side = false) {
        double flops = 0.0, mn = 0.0, tiles64 = 0.0;
        for (const GemmTask& t : gt) {
            // a mirrored (symmetric) result is about half the work: its lower triangle
            const double part = (t.flags & GEMM_MIRROR) ? 0.5 * (1.0 + 1.0 / std::max(1, t.M)) : 1.0;
            for (int q = t.t_begin; q < t.t_end; ++q) flops += part * 2.0 * t.M * t.N * terms[q].K;
            mn += part * double(t.M) * t.N;
            tiles64 += part * double((t.M + 63) / 64) * double((t.N + 63) / 64);
        }
        // tile shape: the autotuned choice for this launch's size bucket; the replay lays out
        // the tiles of the smallest shape, the most of any, so its table bounds every choice
        int variant = 0;
        if (dry) {
            for (int v = 1; v < GEMM_VARIANTS; ++v)
                if (GEMM_SHAPES[v].tm * GEMM_SHAPES[v].tn < GEMM_SHAPES[variant].tm * GEMM_SHAPES[variant].tn)
                    variant = v;
        } else {
            variant = gemm_variant(gemm_bucket(tiles64, mn > 0.0 ? flops / (2.0 * mn) : 0.0), sizeof(R) == 4);
        }
        const GemmShape sh = GEMM_SHAPES[variant];
        for (size_t id = 0; id < gt.size(); ++id) {
            const bool mirror = (gt[id].flags & GEMM_MIRROR) != 0;
            for (int ti = 0; ti * sh.tm < gt[id].M; ++ti)
                for (int tj = 0; tj * sh.tn < gt[id].N; ++tj) {
                    if (mirror && tj * sh.tn >= ti * sh.tm + sh.tm) continue;   // wholly above the diagonal
                    tiles.push_back(GemmTile{int(id), ti, tj, 0});
                }
        }
        if (!tiles.empty()) {
            // the three tables in one upload (one copy on the stream instead of three)
            auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
            const size_t o1 = al(sizeof(GemmTask) * gt.size());
            const size_t o2 = o1 + al(sizeof(GemmTerm) * terms.size());
            std::vector<char> buf(o2 + sizeof(GemmTile) * tiles.size());
            std::memcpy(buf.data(), gt.data(), sizeof(GemmTask) * gt.size());
            std::memcpy(buf.data() + o1, terms.data(), sizeof(GemmTerm) * terms.size());
            std::memcpy(buf.data() + o2, tiles.data(), sizeof(GemmTile) * tiles.size());
            char* dbase = static_cast<char*>(P.stage.upload(buf.data(), buf.size(), P.spool, P.stream));
            GemmTask* dt = reinterpret_cast<GemmTask*>(dbase);
            GemmTerm* dterm = reinterpret_cast<GemmTerm*>(dbase + o1);
            GemmTile* dtile = reinterpret_cast<GemmTile*>(dbase + o2);
            if (!dry) launch_gemm<R>(dt, dterm, dtile, int(tiles.size()), flops, variant, to_side(P, side));
        }
        gt.clear();
        terms.clear();
        tiles.clear();
    }
    void flush_chol(Plan& P, int* d_fail, bool side = false) {
        if (chol.empty()) return;
        for (int big = 0; big < 2; ++big) {       // LDS-resident blocks, then large ones
            std::vector<CholTask> part;
            double flops = 0.0;
            int max_m = 0;
            for (CholTask c : chol) {
                if ((c.m > PIV_LDS_MAX_M) != bool(big)) continue;
                if (big) c.work = P.spool.alloc_n<R>(size_t(c.m) * c.m);
                // potrf m^3/3 + triangular inverse m^3/3 (+ X^T X, m^3/3, in the LDS kernel)
                flops += (big ? 2.0 / 3.0 : 1.0) * double(c.m) * c.m * c.m;
                max_m = std::max(max_m, c.m);
                part.push_back(c);
            }
            if (part.empty()) continue;
            long long* d_stamp = nullptr;
            if (big && trace_pivots) {
                d_stamp = P.spool.alloc_n<long long>(9 * part.size());
                for (size_t q = 0; q < part.size(); ++q) part[q].tstamp = d_stamp + 9 * q;
            }
            CholTask* d = P.stage.upload_vec(part, P.spool, P.stream);
            if (!dry) launch_chol_inv<R>(d, int(part.size()), d_fail, flops, !big, max_m, to_side(P, side));
            if (d_stamp && !dry) {
                if (side) HS_HIP(hipStreamSynchronize(P.side));
                std::vector<long long> h(9 * part.size());
                HS_HIP(hipMemcpy(h.data(), d_stamp, sizeof(long long) * h.size(), hipMemcpyDeviceToHost));
                long long ph[3] = {0, 0, 0}, pp[5] = {0, 0, 0, 0, 0};
                for (size_t q = 0; q < part.size(); ++q) {
                    for (int k = 0; k < 3; ++k) ph[k] = std::max(ph[k], h[9 * q + k + 1] - h[9 * q + k]);
                    for (int k = 0; k < 5; ++k) pp[k] = std::max(pp[k], h[9 * q + 4 + k]);
                }
                std::fprintf(stderr,
                             "    pivot batch n=%zu max_m=%d kcycles copy %lld chol %lld trinv %lld | panel: copy %lld "
                             "l11 %lld l21 %lld wb %lld trail %lld\n",
                             part.size(), max_m, ph[0] / 1000, ph[1] / 1000, ph[2] / 1000, pp[0] / 1000, pp[1] / 1000,
                             pp[2] / 1000, pp[3] / 1000, pp[4] / 1000);
            }
            if (big) {      // A^{-1} = X^T X, X = L^{-1} left in the work matrices
                for (const CholTask& c : part)
                    gemm(static_cast<R*>(c.Ainv), c.ldi, c.m, c.m, 1.0, 0.0, static_cast<const R*>(c.work), c.m, 1,
                         static_cast<const R*>(c.work), c.m, 0, c.m);
                flush_gemm(P, side);
            }
        }
        chol.clear();
    }
};

template <typename R>
size_t blk_bytes(int r, int c) { return ((size_t(r) * c * sizeof(R)) + 255) & ~size_t(255); }

}  // namespace

// Compression tolerance of the super nodes of depth d (§7.1, "3D cases", Table 3). The
// first super-node depth lmax = L - 1 is the leaf level of the schedules.
//   HSOLVE_EPS_CONSTANT  eps on every level;
//   HSOLVE_EPS_SHRINK    eps 2^{(d - lmax)/3}: eps at the leaves, smaller toward the root
//                        (the paper's adaptive GC choice);
//   HSOLVE_EPS_GROW      eps h 2^{(lmax - d)/3} with h = n^{-1/dim}: small at the leaves,
//                        larger toward the root (the paper's adaptive LoRaSp choice).
double level_eps(const Plan& P, int d) {
    const double eps = P.opt.eps;
    const int lmax = std::max(P.L - 1, 0);
    switch (P.opt.eps_schedule) {
        case HSOLVE_EPS_SHRINK: return eps * std::exp2((d - lmax) / 3.0);
        case HSOLVE_EPS_GROW: {
            const double h = std::pow(double(P.n), -1.0 / std::max(1, P.opt.dim));
            return eps * h * std::exp2((lmax - d) / 3.0);
        }
        default: return eps;
    }
}

// The factorization in the storage type R: double (factor_prec = 64), or float
// (factor_prec = 32: blocks, factors, pivots and GEMMs in FP32 on the matrix cores; the Gram
// matrices and kept vectors are promoted to FP64 for the symmetric eigen-solver and its basis
// is rounded back to FP32 after the orthonormalisation).
template <typename R>
static void factor_t(Plan& P, const double* values_in) {
    constexpr bool F32 = std::is_same<R, float>::value;
    using clk = std::chrono::steady_clock;
    auto gm = [](const NodeNum& nn) { return static_cast<R*>(nn.Gm); };
    const auto t0 = clk::now();
    const bool dry = P.dry;
    hipStream_t st = P.stream;
    const int L = P.L;
    const int nlev = std::max(L, 1);
    // GC_PROJ1 is GC whose kept vectors are first truncated (Appendix B); the compression
    // kernels then run the GC path
    const bool proj1 = P.opt.variant == HSOLVE_GC_PROJ1 && P.opt.eps1 > 0.0;
    const bool gc = P.opt.variant == HSOLVE_GC || P.opt.variant == HSOLVE_GC_PROJ1;
    const int cmp_variant = gc ? HSOLVE_GC : HSOLVE_LORASP;
    const int p = P.nphi;
    const int q_gc = gc ? 2 * p : 0;   // columns of [phi_s, A_sw phi_w]
    const bool overlap = P.opt.overlap_pivots != 0 && !dry;
    const int max_super = P.opt.max_super;

    P.factored = false;
    P.d_V = nullptr;
    P.d_X = nullptr;
    P.V_cols = 0;
    P.d_krylov = nullptr;
    P.krylov_cols = 0;
    P.d_gmres = nullptr;          // the GMRES basis lived in the workspace that is reset below
    P.gmres_restart = 0;
    P.sched.clear();
    if (!dry) {
        clear_graphs(P);      // they replay the previous factorization's schedule
        if (!P.side) {      // second stream for the pivot blocks (default priority)
            HS_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
            HS_HIP(hipEventCreateWithFlags(&P.ev_ready, hipEventDisableTiming));
            HS_HIP(hipEventCreateWithFlags(&P.ev_done, hipEventDisableTiming));
        }
        if (!P.side2) {     // third stream for the large nodes' compression (default priority)
            HS_HIP(hipStreamCreateWithFlags(&P.side2, hipStreamNonBlocking));
            HS_HIP(hipEventCreateWithFlags(&P.ev_ready2, hipEventDisableTiming));
            HS_HIP(hipEventCreateWithFlags(&P.ev_done2, hipEventDisableTiming));
        }
        if (!P.h_flags)
            HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_flags), sizeof(int) * (size_t(4) << nlev) + 64,
                                 hipHostMallocDefault));
        HS_HIP(hipStreamSynchronize(P.side));
        HS_HIP(hipStreamSynchronize(P.side2));
        HS_HIP(hipStreamSynchronize(st));
        // host or device values (unified addressing decides the direction)
        HS_HIP(hipMemcpyAsync(P.d_values, values_in, size_t(P.nnz) * sizeof(double), hipMemcpyDefault, st));
    }
    int* d_bad = P.fpool.alloc_n<int>(1);
    if (!dry) {
        launch_check_finite(P.d_values, P.nnz, d_bad, st);
        HS_HIP(hipMemcpyAsync(P.h_flags, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HS_HIP(hipStreamSynchronize(st));
        if (P.h_flags[0]) throw Error{HSOLVE_ERR_INVALID, "matrix values contain NaN or Inf"};
    }
    P.stage.reset();
    P.stage.dry = dry;
    P.lpool[0].reset();
    P.lpool[1].reset();
    P.spool.reset();

    P.num.assign(nlev, LevelNum{});
    Live lives[2];
    std::vector<std::vector<R*>> phi_sup(nlev), phi_red(nlev);
    double flops = 0.0;
    int max_rank = 0;
    int* h_flags = P.h_flags;   // fail flags of the level + ranks of the colour

    const bool trace = !dry && std::getenv("HSOLVE_TRACE") != nullptr;
    auto now_ms = [&] { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); };
    for (int d = nlev - 1; d >= 0; --d) {
        const LevelSym& S = P.sym[d];
        const int nd = 1 << d;
        LevelNum& LN = P.num[d];
        LN.msz.assign(nd, 0);
        LN.ksz.assign(nd, 0);
        LN.node.assign(nd, NodeNum{});
        const bool first = (d == nlev - 1);
        for (int s = 0; s < nd; ++s) {
            if (!S.super_nonempty[s]) continue;
            if (L == 0) LN.msz[s] = P.n;
            else if (first) LN.msz[s] = P.leaf_off[2 * s + 2] - P.leaf_off[2 * s];
            else LN.msz[s] = P.num[d + 1].ksz[2 * s] + P.num[d + 1].ksz[2 * s + 1];
            if (LN.msz[s] > max_super) {
                // the replay bounds the merged size by the cap; a factorization that exceeds it
                // stops here (its arena and kernels were sized for max_super)
                if (dry) LN.msz[s] = max_super;
                else {
                    P.stats.fail_level = d;
                    P.stats.fail_node = s;
                    throw Error{HSOLVE_ERR_TOO_LARGE,
                                "super node of " + std::to_string(LN.msz[s]) + " unknowns at depth " +
                                    std::to_string(d) + " exceeds max_super = " + std::to_string(max_super)};
                }
            }
        }
        const double eps = level_eps(P, d);
        Live& live = lives[d & 1];
        live.map.clear();
        Region& lp = P.lpool[d & 1];
        lp.reset();
        phi_sup[d].assign(nd, nullptr);
        phi_red[d].assign(nd, nullptr);
        P.spool.reset();
        int* d_fail = lp.alloc_n<int>(nd);
        if (!dry) HS_HIP(hipMemsetAsync(d_fail, 0, sizeof(int) * nd, st));
        Batch<R> B;
        B.trace_pivots = trace;
        B.dry = dry;

        // ---- blocks of the level at its start: diagonal + upper partners, one zeroed region
        size_t region = 0;
        for (int s = 0; s < nd; ++s) {
            if (!S.super_nonempty[s]) continue;
            region += blk_bytes<R>(LN.msz[s], LN.msz[s]);
            for (int j : S.init_partners[s])
                if (j > s) region += blk_bytes<R>(LN.msz[s], LN.msz[j]);
        }
        char* base = static_cast<char*>(lp.alloc(region));
        if (!dry) launch_fill<R>(reinterpret_cast<R*>(base), R(0), int64_t(region / sizeof(R)), st);
        std::vector<int32_t> blk_begin(nd + 1, 0), blk_col, blk_ld;
        std::vector<void*> blk_ptr;
        {
            size_t off = 0;
            for (int s = 0; s < nd; ++s) {
                blk_begin[s] = int32_t(blk_col.size());
                if (!S.super_nonempty[s]) continue;
                const int m = LN.msz[s];
                Block b{base + off, m, m, m};
                off += blk_bytes<R>(m, m);
                live.put(s, s, b);
                blk_col.push_back(s); blk_ld.push_back(m); blk_ptr.push_back(b.p);
                for (int j : S.init_partners[s]) {
                    if (j <= s) continue;
                    Block c{base + off, m, LN.msz[j], m};
                    off += blk_bytes<R>(m, LN.msz[j]);
                    live.put(s, j, c);
                    blk_col.push_back(j); blk_ld.push_back(m); blk_ptr.push_back(c.p);
                }
            }
            blk_begin[nd] = int32_t(blk_col.size());
        }
        if (first) {
            std::vector<int32_t> super_first(nd, 0);
            if (L > 0)
                for (int s = 0; s < nd; ++s) super_first[s] = P.leaf_off[2 * s];
            const int32_t* d_sf = P.stage.upload_vec(super_first, P.spool, st);
            void* const* d_bp = P.stage.upload_vec(blk_ptr, P.spool, st);
            const int32_t* d_bl = P.stage.upload_vec(blk_ld, P.spool, st);
            const int32_t* d_bc = P.stage.upload_vec(blk_col, P.spool, st);
            const int32_t* d_bb = P.stage.upload_vec(blk_begin, P.spool, st);
            if (!dry)
                launch_leaf_scatter<R>(P.d_row_ptr, P.d_col_idx, P.d_values, P.d_iperm, P.d_pos_super, d_sf, d_bp,
                                    d_bl, d_bc, d_bb, P.n, st);
            if (gc) {
                std::vector<R> h(size_t(P.n) * p);
                size_t off = 0;
                std::vector<size_t> node_off(nd, 0);
                for (int s = 0; s < nd; ++s) {
                    node_off[s] = off;
                    const int m = LN.msz[s];
                    const int p0 = (L == 0) ? 0 : P.leaf_off[2 * s];
                    for (int c = 0; c < p; ++c)
                        for (int i = 0; i < m; ++i)
                            h[off + size_t(c) * m + i] = R(P.phi[size_t(P.perm[p0 + i]) + size_t(c) * P.n]);
                    off += size_t(m) * p;
                }
                R* dphi = P.stage.upload_vec(h, lp, st);
                for (int s = 0; s < nd; ++s) phi_sup[d][s] = dphi + node_off[s];
            }
        } else {
            Live& prev = lives[(d + 1) & 1];
            const std::vector<int>& kc = P.num[d + 1].ksz;
            for (int I = 0; I < nd; ++I) {
                if (!S.super_nonempty[I]) continue;
                std::vector<int> Js{I};
                for (int j : S.init_partners[I])
                    if (j > I) Js.push_back(j);
                for (int J : Js) {
                    Block* C = live.find(I, J);
                    for (int a = 0; a < 2; ++a) {
                        const int ca = 2 * I + a, ka = kc[ca];
                        if (!ka) continue;
                        const int roff = a ? kc[2 * I] : 0;
                        for (int b = 0; b < 2; ++b) {
                            const int cb = 2 * J + b, kb = kc[cb];
                            if (!kb || (I == J && a > b)) continue;
                            const int coff = b ? kc[2 * J] : 0;
                            Block* ch = prev.find(ca, cb);
                            if (!ch) continue;
                            B.copy(static_cast<R*>(ch->p), ch->ld, static_cast<R*>(C->p) + roff + size_t(coff) * C->ld,
                                   C->ld, ch->rows, ch->cols, 0);
                            if (I == J && a == 0 && b == 1)
                                B.copy(static_cast<R*>(ch->p), ch->ld, static_cast<R*>(C->p) + kc[2 * I], C->ld, ch->cols,
                                       ch->rows, 1);
                        }
                    }
                }
                if (gc) {
                    const int m = LN.msz[I];
                    R* f = lp.alloc_n<R>(size_t(m) * p);
                    phi_sup[d][I] = f;
                    int r0 = 0;
                    for (int a = 0; a < 2; ++a) {
                        const int ka = kc[2 * I + a];
                        if (!ka) continue;
                        B.copy(phi_red[d + 1][2 * I + a], ka, f + r0, m, ka, p, 0);
                        r0 += ka;
                    }
                }
            }
            B.flush_copies(P);
        }

        // ---- colours
        auto cursize = [&](int j, bool red) { return red ? LN.ksz[j] : LN.msz[j]; };
        for (size_t c = 0; c < S.colours.size(); ++c) {
            const std::vector<int>& nodes = S.colours[c];
            P.spool.reset();    // stream order: the previous colour's kernels run first
            const double tc0 = trace ? now_ms() : 0.0;
            // --- pivot blocks: Cholesky and inverse of every A_ss of the colour on the side
            // stream, overlapped with the compression below (which does not read A_ss); the
            // inverses land in Ainv (ld m) and join the plan's stream in phase B
            std::vector<R*> Ainv(nodes.size(), nullptr);
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                const int m = LN.msz[s];
                Block* dg = live.find(s, s);
                if (!dg) throw Error{HSOLVE_ERR_DEVICE, "internal: missing diagonal block"};
                Ainv[q] = P.spool.alloc_n<R>(size_t(m) * m);
                B.chol.push_back(CholTask{dg->p, Ainv[q], nullptr, nullptr, dg->ld, m, m, s});
                flops += double(m) * m * m;      // Cholesky (m^3/3) + inverse (2m^3/3)
            }
            B.flush_chol(P, d_fail, overlap);
            if (overlap) HS_HIP(hipEventRecord(P.ev_done, P.side));
            // --- phase A: compression of the nodes with well-separated blocks
            // Asw: the gathered A_sw (R); U: the basis in double from the eigen-solver, Ur: the
            // basis the elimination uses (R; the same buffer in FP64)
            struct CompNode { int s, slot, wt; R* Asw; double* U; R* Ur; };
            std::vector<PromoteTask> promote;
            std::vector<CompNode> comp;
            std::vector<CompressTask> ctasks;
            for (int s : nodes) {
                if (S.W[s].empty()) continue;
                const int m = LN.msz[s];
                int wt = 0;
                for (size_t t = 0; t < S.W[s].size(); ++t) wt += cursize(S.W[s][t], S.Wred[s][t]);
                R* Asw = P.spool.alloc_n<R>(size_t(m) * wt);
                R* G = P.spool.alloc_n<R>(size_t(m) * m);
                double* U = P.spool.alloc_n<double>(size_t(m) * m);
                double* work = P.spool.alloc_n<double>(cmp_work_doubles(m));
                R* Z = nullptr;
                int off = 0;
                for (size_t t = 0; t < S.W[s].size(); ++t) {
                    const int w = S.W[s][t];
                    const int ws = cursize(w, S.Wred[s][t]);
                    Block* b = live.find(s, w);
                    if (!b) throw Error{HSOLVE_ERR_DEVICE, "internal: missing well-separated block"};
                    if (s < w) B.copy(static_cast<R*>(b->p), b->ld, Asw + size_t(off) * m, m, m, ws, 0);
                    else B.copy(static_cast<R*>(b->p), b->ld, Asw + size_t(off) * m, m, m, ws, 1);
                    off += ws;
                }
                if (gc) {
                    R* phiW = P.spool.alloc_n<R>(size_t(wt) * p);
                    int r0 = 0;
                    for (size_t t = 0; t < S.W[s].size(); ++t) {
                        const int w = S.W[s][t];
                        const bool red = S.Wred[s][t];
                        const int ws = cursize(w, red);
                        B.copy(red ? phi_red[d][w] : phi_sup[d][w], ws, phiW + r0, wt, ws, p, 0);
                        r0 += ws;
                    }
                    Z = P.spool.alloc_n<R>(size_t(m) * 2 * p);
                    B.copy(phi_sup[d][s], m, Z, m, m, p, 0);
                    B.gemm(Z + size_t(p) * m, m, m, p, 1.0, 0.0, Asw, m, 0, phiW, wt, 0, wt);
                    flops += 2.0 * m * wt * p;
                }
                B.gemm_sym(G, m, m, 1.0, Asw, m, 0, wt);
                flops += double(m) * (m + 1) * wt;
                const int slot = int(comp.size());
                const double* Gd = reinterpret_cast<const double*>(G);
                const double* Zd = reinterpret_cast<const double*>(Z);
                if constexpr (F32) {      // the eigen-solver reads FP64
                    double* g64 = P.spool.alloc_n<double>(size_t(m) * m);
                    promote.push_back(PromoteTask{G, g64, (long long)m * m});
                    Gd = g64;
                    if (Z) {
                        double* z64 = P.spool.alloc_n<double>(size_t(m) * 2 * p);
                        promote.push_back(PromoteTask{Z, z64, (long long)m * 2 * p});
                        Zd = z64;
                    }
                }
                comp.push_back(CompNode{s, slot, wt, Asw, U, nullptr});
                ctasks.push_back(CompressTask{Gd, Zd, work, U, nullptr, m, gc ? 2 * p : 0, wt, slot});
            }
            // kept count per node, then (with the refinement) the extra eigenvectors computed past it
            const bool ritz = !F32 && eps > 0.0 && P.opt.cmp_ritz != 0;
            int* d_rank = P.spool.alloc_n<int>(2 * std::max<size_t>(1, comp.size()));
            int* d_extra = ritz ? d_rank + comp.size() : nullptr;
            long long* d_stamp = nullptr;
            if (trace && !ctasks.empty()) {
                d_stamp = P.spool.alloc_n<long long>(16 * ctasks.size());
                HS_HIP(hipMemsetAsync(d_stamp, 0, sizeof(long long) * 16 * ctasks.size(), st));
                for (size_t q2 = 0; q2 < ctasks.size(); ++q2) ctasks[q2].tstamp = d_stamp + 16 * q2;
            }
            B.flush_copies(P);
            B.flush_gemm(P);
            if (!promote.empty()) {
                double elems = 0.0;
                for (const PromoteTask& t : promote) elems += double(t.count);
                const PromoteTask* d_pr = P.stage.upload_vec(promote, P.spool, st);
                if (!dry) launch_promote(d_pr, int(promote.size()), elems, st);
            }
            if (proj1 && !ctasks.empty()) {
                const CompressTask* d_all = P.stage.upload_vec(ctasks, P.spool, st);
                if (!dry) launch_gc_truncate(d_all, int(ctasks.size()), P.opt.eps1, st);
            }
            // The nodes held in LDS and the larger ones are two independent launch chains. With
            // overlap the larger nodes' chain runs on the third stream beside the other: both
            // tables are uploaded first, that stream waits for everything enqueued so far (Gram
            // matrices, GC bases, tables), and the plan's stream waits for it before the ranks
            // are read back.
            struct Part { std::vector<CompressTask> t; double flops = 0.0; int max_m = 0; };
            Part parts[2];
            for (const CompressTask& ct : ctasks) {
                Part& pt = parts[ct.m > LDS_MAX_M ? 1 : 0];
                // counted work of the reduction kernel: one Householder tridiagonalisation,
                // 4/3 m^3 (two when GC keeps more than four vectors)
                const double m3 = double(ct.m) * ct.m * ct.m;
                pt.flops += ((gc && ct.nz > 4) ? 8.0 / 3.0 : 4.0 / 3.0) * m3;
                pt.max_m = std::max(pt.max_m, ct.m);
                pt.t.push_back(ct);
            }
            const CompressTask* d_part[2] = {nullptr, nullptr};
            for (int big = 0; big < 2; ++big)
                if (!parts[big].t.empty()) d_part[big] = P.stage.upload_vec(parts[big].t, P.spool, st);
            const bool two = overlap && !parts[0].t.empty() && !parts[1].t.empty();
            if (!dry) {
                if (two) {
                    HS_HIP(hipEventRecord(P.ev_ready2, st));
                    HS_HIP(hipStreamWaitEvent(P.side2, P.ev_ready2, 0));
                }
                for (int big = 0; big < 2; ++big) {
                    const Part& pt = parts[big];
                    if (pt.t.empty()) continue;
                    launch_compress(d_part[big], int(pt.t.size()), cmp_variant, eps, d_rank, d_extra,
                                    ritz ? RITZ_EXTRA : 0, pt.flops, !big, pt.max_m, P.opt.cmp_lpe,
                                    P.opt.cmp_vectors, (two && big) ? P.side2 : st);
                }
                if (two) {
                    HS_HIP(hipEventRecord(P.ev_done2, P.side2));
                    HS_HIP(hipStreamWaitEvent(st, P.ev_done2, 0));
                }
            }
            // The contributions to the Schur complement of phase B, gathered per target block:
            // targets in ascending key order, the contributions to one target in node order (a
            // stable sort of one flat list). They depend on the schedule only, so the host
            // sorts them while the compression runs.
            struct Contrib { uint64_t key; int q, a, b; };
            std::vector<Contrib> contribs;
            for (size_t q = 0; q < nodes.size(); ++q) {
                const std::vector<int>& Nl = S.N[nodes[q]];
                for (size_t a = 0; a < Nl.size(); ++a)
                    for (size_t b = a; b < Nl.size(); ++b)
                        contribs.push_back(Contrib{bkey(Nl[a], Nl[b]), int(q), int(a), int(b)});
            }
            std::stable_sort(contribs.begin(), contribs.end(),
                             [](const Contrib& x, const Contrib& y) { return x.key < y.key; });
            if (!dry) {
                // the pivot blocks of this colour may still run on the side stream: their failure
                // flags are read only after it has finished (the compression keeps overlapping)
                if (overlap) HS_HIP(hipStreamWaitEvent(st, P.ev_done, 0));
                HS_HIP(hipMemcpyAsync(h_flags, d_fail, sizeof(int) * nd, hipMemcpyDeviceToHost, st));
                if (!comp.empty())
                    HS_HIP(hipMemcpyAsync(h_flags + nd, d_rank, sizeof(int) * comp.size() * (ritz ? 2 : 1),
                                          hipMemcpyDeviceToHost, st));
                HS_HIP(hipStreamSynchronize(st));
                P.stage.reset();
                for (int s = 0; s < nd; ++s)
                    if (h_flags[s]) {
                        P.stats.fail_level = d;
                        P.stats.fail_node = s;
                        throw Error{HSOLVE_ERR_NOT_SPD, "pivot block not positive definite"};
                    }
            }
            std::vector<int> kxs(comp.size(), 0);
            for (const CompNode& cn : comp) {
                // the replay takes the largest rank the compression can return:
                // |U1| + k2 <= min(m, 2p + |W|) (R5: at least one column)
                const int k = dry ? std::max(1, std::min(LN.msz[cn.s], q_gc + cn.wt)) : h_flags[nd + cn.slot];
                if (k < 0 || k > LN.msz[cn.s])
                    throw Error{HSOLVE_ERR_DEVICE,
                                "eigen-solver did not converge (level " + std::to_string(d) + ", node " +
                                    std::to_string(cn.s) + ", m " + std::to_string(LN.msz[cn.s]) +
                                    ", |W| " + std::to_string(cn.wt) + ", k " + std::to_string(k) + ")"};
                LN.ksz[cn.s] = k;
                max_rank = std::max(max_rank, k);
                if (ritz) {
                    const int kx = dry ? std::min(RITZ_EXTRA, LN.msz[cn.s] - k)
                                       : h_flags[nd + comp.size() + cn.slot];
                    if (kx < 0 || k + kx > LN.msz[cn.s])
                        throw Error{HSOLVE_ERR_DEVICE, "internal: extra eigenvectors out of range"};
                    kxs[cn.slot] = kx;
                }
            }
            double tc1 = 0.0;
            std::vector<long long> stamps;
            if (trace) {
                tc1 = now_ms();
                if (d_stamp) {
                    stamps.resize(16 * ctasks.size());
                    HS_HIP(hipMemcpy(stamps.data(), d_stamp, sizeof(long long) * stamps.size(),
                                     hipMemcpyDeviceToHost));
                }
            }
            // The eigenvectors of nearly equal eigenvalues come from independent inverse
            // iterations and are orthogonal only to about u ||G|| / gap. One Newton-Schulz step
            // towards the polar factor, U <- U (3 I - U^T U) / 2, restores U^T U = I to second
            // order on the matrix cores; it keeps span(U), so the GC vectors stay in it.
            {
                // in double: the eigen-solver's basis (for FP32, rounded once afterwards)
                Batch<double> Bd;
                Batch<double>& B64 = [&]() -> Batch<double>& {
                    if constexpr (F32) return Bd;
                    else return B;
                }();
                Bd.dry = dry;
                // (with the refinement the extra eigenvectors join the step: the window below
                // must be orthonormal as a whole)
                std::vector<double*> Wsc(comp.size(), nullptr);
                for (CompNode& cn : comp) {
                    const int m = LN.msz[cn.s], k = LN.ksz[cn.s] + kxs[cn.slot];
                    if (k < 2) continue;
                    Wsc[cn.slot] = P.spool.alloc_n<double>(size_t(k) * k);
                    B64.gemm(Wsc[cn.slot], k, k, k, 1.0, 0.0, cn.U, m, 1, cn.U, m, 0, m);
                    flops += 2.0 * m * k * k;
                }
                B64.flush_gemm(P);
                for (CompNode& cn : comp) {
                    const int m = LN.msz[cn.s], k = LN.ksz[cn.s] + kxs[cn.slot];
                    if (k < 2) continue;
                    double* Un = P.spool.alloc_n<double>(size_t(m) * k);
                    B64.copy(cn.U, m, Un, m, m, k, 0);
                    B64.gemm(Un, m, m, k, -0.5, 1.5, cn.U, m, 0, Wsc[cn.slot], k, 0, k);
                    flops += 2.0 * m * k * k;
                    cn.U = Un;
                }
                B64.flush_copies(P);
                B64.flush_gemm(P);
                // Rayleigh-Ritz on the window W of the last kept directions and the extra ones
                // (w + kx <= RITZ_MAX columns): the eigenvectors of C = (W^T A_sw)(W^T A_sw)^T
                // rotate W, and the first w replace the kept ones. The eigenvectors of the Gram
                // matrix separate two singular values sigma_k > eps sigma_1 > sigma_k+1 only to
                // about u sigma_1 / (2 eps (sigma_k - sigma_k+1)); C's entries carry errors of
                // u sigma_1 sigma_k, which resolves the pair to u sigma_1 / (sigma_k - sigma_k+1),
                // the accuracy of an SVD of A_sw itself.
                if constexpr (!F32) {
                    if (ritz) {
                        struct Win { double* W; const double* A; double* Bw; int m, wt, w, s; };
                        std::vector<Win> win;
                        for (CompNode& cn : comp) {
                            const int m = LN.msz[cn.s], k = LN.ksz[cn.s], kx = kxs[cn.slot];
                            // window: kept directions past the GC vectors (at most q_gc of them)
                            const int w = std::min(RITZ_KEEP, k - q_gc);
                            if (!dry && (kx <= 0 || w <= 0)) continue;
                            // the replay counts every node at the largest window
                            const int ss = dry ? std::min(RITZ_MAX, m) : w + kx;
                            Win x{cn.U + (dry ? size_t(0) : size_t(k - w) * m), reinterpret_cast<const double*>(cn.Asw),
                                  P.spool.alloc_n<double>(size_t(ss) * cn.wt), m, cn.wt, dry ? 0 : w, ss};
                            win.push_back(x);
                        }
                        std::vector<RitzTask> rt;
                        for (const Win& x : win) {
                            B64.gemm(x.Bw, x.s, x.s, x.wt, 1.0, 0.0, x.W, x.m, 1, x.A, x.m, 0, x.m);
                            flops += 2.0 * x.s * x.m * x.wt;
                            rt.push_back(RitzTask{x.Bw, x.W, x.s, x.w, x.wt, x.m, x.m});
                        }
                        B64.flush_gemm(P);
                        if (!rt.empty()) {
                            const RitzTask* d_rt = P.stage.upload_vec(rt, P.spool, st);
                            if (!dry) launch_comp_ritz(d_rt, int(rt.size()), st);
                        }
                    }
                }
                if constexpr (F32) {
                    std::vector<DemoteTask> dt;
                    double elems = 0.0;
                    for (CompNode& cn : comp) {
                        const int m = LN.msz[cn.s], k = LN.ksz[cn.s];
                        if (!k) continue;
                        cn.Ur = P.spool.alloc_n<R>(size_t(m) * k);
                        dt.push_back(DemoteTask{cn.U, reinterpret_cast<float*>(cn.Ur), (long long)m * k});
                        elems += double(m) * k;
                    }
                    if (!dt.empty()) {
                        const DemoteTask* d_dt = P.stage.upload_vec(dt, P.spool, st);
                        if (!dry) launch_demote(d_dt, int(dt.size()), elems, st);
                    }
                } else {
                    for (CompNode& cn : comp) cn.Ur = reinterpret_cast<R*>(cn.U);
                }
            }
            std::vector<const CompNode*> compof(nd, nullptr);
            for (const CompNode& cn : comp) compof[cn.s] = &cn;

            // --- phase B: elimination
            std::vector<R*> AN(nodes.size()), Ysc(nodes.size());
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                nn.m = LN.msz[s];
                nn.k = LN.ksz[s];
                nn.ka = (first && L > 0) ? (P.leaf_off[2 * s + 1] - P.leaf_off[2 * s])
                                         : (first ? nn.m : P.num[d + 1].ksz[2 * s]);
                nn.ntot = 0;
                nn.noff.clear();
                for (size_t t = 0; t < S.N[s].size(); ++t) {
                    nn.noff.push_back(nn.ntot);
                    nn.ntot += cursize(S.N[s][t], S.Nred[s][t]);
                }
                nn.ldG = nn.m + nn.ntot + nn.k;
                nn.Gm = P.fpool.alloc_n<R>(size_t(nn.ldG) * nn.m);
                const int m = nn.m;
                AN[q] = nn.ntot ? P.spool.alloc_n<R>(size_t(nn.ntot) * m) : nullptr;
                for (size_t t = 0; t < S.N[s].size(); ++t) {
                    const int nb = S.N[s][t];
                    const int ns = cursize(nb, S.Nred[s][t]);
                    Block* b = live.find(nb, s);
                    if (!b) throw Error{HSOLVE_ERR_DEVICE, "internal: missing neighbour block"};
                    if (nb < s) B.copy(static_cast<R*>(b->p), b->ld, AN[q] + nn.noff[t], nn.ntot, ns, m, 0);
                    else B.copy(static_cast<R*>(b->p), b->ld, AN[q] + nn.noff[t], nn.ntot, ns, m, 1);
                }
                B.copy(Ainv[q], m, gm(nn), nn.ldG, m, m, 0);      // A_ss^-1 into rows 0..m-1 of Gm
            }
            B.flush_copies(P);
            // Y = A_ss^-1 U, S = U^T Y
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                if (!nn.k) continue;
                Ysc[q] = P.spool.alloc_n<R>(size_t(nn.m) * nn.k);
                B.gemm(Ysc[q], nn.m, nn.m, nn.k, 1.0, 0.0, gm(nn), nn.ldG, 0, compof[s]->Ur, nn.m, 0, nn.m);
                flops += 2.0 * nn.m * nn.m * nn.k;
            }
            B.flush_gemm(P);
            std::vector<R*> Ssc(nodes.size()), Sinv(nodes.size());
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                if (!nn.k) continue;
                Ssc[q] = P.spool.alloc_n<R>(size_t(nn.k) * nn.k);
                B.gemm(Ssc[q], nn.k, nn.k, nn.k, 1.0, 0.0, compof[s]->Ur, nn.m, 1, Ysc[q], nn.m, 0, nn.m);
                flops += 2.0 * nn.m * nn.k * nn.k;
            }
            B.flush_gemm(P);
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                if (!nn.k) continue;
                Sinv[q] = static_cast<R*>(lp.alloc(blk_bytes<R>(nn.k, nn.k)));
                B.chol.push_back(CholTask{Ssc[q], Sinv[q], nullptr, nullptr, nn.k, nn.k, nn.k, s});
                flops += double(nn.k) * nn.k * nn.k;
            }
            B.flush_chol(P, d_fail);
            // P_ss = S^-1 Y^T (rows m+ntot.. of Gm)
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                if (!nn.k) continue;
                B.gemm(gm(nn) + nn.m + nn.ntot, nn.ldG, nn.k, nn.m, 1.0, 0.0, Sinv[q], nn.k, 0, Ysc[q],
                       nn.m, 1, nn.k);
                flops += 2.0 * nn.k * nn.k * nn.m;
            }
            B.flush_gemm(P);
            // M_ss = A_ss^-1 - Y P_ss; exactly zero when U is square (Appendix A)
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                if (!nn.k) continue;
                if (nn.k == nn.m) {
                    B.open(gm(nn), nn.ldG, nn.m, nn.m, 0.0, 0.0);
                    B.close();
                    continue;
                }
                B.gemm(gm(nn), nn.ldG, nn.m, nn.m, -1.0, 1.0, Ysc[q], nn.m, 0, gm(nn) + nn.m + nn.ntot,
                       nn.ldG, 0, nn.k);
                flops += 2.0 * nn.m * nn.m * nn.k;
            }
            B.flush_gemm(P);
            // T_N = A_Ns M_ss; red-node blocks L_nr = A_ns P_ss^T, R, S^-1; phi_r = U^T phi_s
            for (size_t q = 0; q < nodes.size(); ++q) {
                const int s = nodes[q];
                NodeNum& nn = LN.node[s];
                const int m = nn.m, k = nn.k;
                if (nn.ntot) {
                    B.gemm(gm(nn) + m, nn.ldG, nn.ntot, m, 1.0, 0.0, AN[q], nn.ntot, 0, gm(nn), nn.ldG, 0, m);
                    flops += 2.0 * nn.ntot * m * m;
                }
                if (!k) {
                    for (int j : S.N[s]) live.erase(s, j);
                    for (int j : S.W[s]) live.erase(s, j);
                    live.erase(s, s);
                    continue;
                }
                const R* Pm = gm(nn) + m + nn.ntot;
                for (size_t t = 0; t < S.N[s].size(); ++t) {
                    const int nb = S.N[s][t];
                    const int ns = cursize(nb, S.Nred[s][t]);
                    if (nb < s) {
                        R* blk = static_cast<R*>(lp.alloc(blk_bytes<R>(ns, k)));
                        live.put(nb, s, Block{blk, ns, k, ns});
                        B.gemm(blk, ns, ns, k, 1.0, 0.0, AN[q] + nn.noff[t], nn.ntot, 0, Pm, nn.ldG, 1, m);
                    } else {
                        R* blk = static_cast<R*>(lp.alloc(blk_bytes<R>(k, ns)));
                        live.put(s, nb, Block{blk, k, ns, k});
                        B.gemm(blk, k, k, ns, 1.0, 0.0, Pm, nn.ldG, 0, AN[q] + nn.noff[t], nn.ntot, 1, m);
                    }
                    flops += 2.0 * ns * m * k;
                }
                const CompNode* cn = compof[s];
                int off = 0;
                for (size_t t = 0; t < S.W[s].size(); ++t) {
                    const int w = S.W[s][t];
                    const int ws = cursize(w, S.Wred[s][t]);
                    const R* Aw = cn->Asw + size_t(off) * m;
                    if (s < w) {
                        R* blk = static_cast<R*>(lp.alloc(blk_bytes<R>(k, ws)));
                        live.put(s, w, Block{blk, k, ws, k});
                        B.gemm(blk, k, k, ws, 1.0, 0.0, cn->Ur, m, 1, Aw, m, 0, m);
                    } else {
                        R* blk = static_cast<R*>(lp.alloc(blk_bytes<R>(ws, k)));
                        live.put(w, s, Block{blk, ws, k, ws});
                        B.gemm(blk, ws, ws, k, 1.0, 0.0, Aw, m, 1, cn->Ur, m, 0, m);
                    }
                    flops += 2.0 * ws * m * k;
                    off += ws;
                }
                live.put(s, s, Block{Sinv[q], k, k, k});
                if (gc) {
                    R* f = lp.alloc_n<R>(size_t(k) * p);
                    phi_red[d][s] = f;
                    B.gemm(f, k, k, p, 1.0, 0.0, cn->Ur, m, 1, phi_sup[d][s], m, 0, m);
                }
            }
            B.flush_gemm(P);
            // Schur complement on the neighbours, gathered per target block (contribs)
            for (size_t i0 = 0, i1 = 0; i0 < contribs.size(); i0 = i1) {
                const uint64_t key = contribs[i0].key;
                for (i1 = i0 + 1; i1 < contribs.size() && contribs[i1].key == key; ++i1) {}
                const int a = int(key >> 32), b = int(key & 0xffffffffu);
                const Contrib& first = contribs[i0];
                const int s0 = nodes[first.q];
                const int sa = cursize(a, S.Nred[s0][first.a]);
                const int sb = cursize(b, S.Nred[s0][first.b]);
                Block* C = live.find(a, b);
                bool fresh = false;
                if (!C) {
                    R* blk = static_cast<R*>(lp.alloc(blk_bytes<R>(sa, sb)));
                    live.put(a, b, Block{blk, sa, sb, sa});
                    C = live.find(a, b);
                    fresh = true;
                }
                B.open(static_cast<R*>(C->p), C->ld, sa, sb, -1.0, fresh ? 0.0 : 1.0);
                for (size_t i = i0; i < i1; ++i) {
                    const Contrib& ct = contribs[i];
                    const NodeNum& nn = LN.node[nodes[ct.q]];
                    B.term(gm(nn) + nn.m + nn.noff[ct.a], nn.ldG, 0, AN[ct.q] + nn.noff[ct.b], nn.ntot, 1,
                           nn.m);
                    flops += 2.0 * sa * sb * nn.m;
                }
                B.close();
            }
            B.flush_gemm(P);
            if (trace) {
                HS_HIP(hipStreamSynchronize(st));
                int mm = 0, mw = 0, mk = 0;
                for (int s2 : nodes) {
                    mm = std::max(mm, LN.msz[s2]);
                    mk = std::max(mk, LN.ksz[s2]);
                }
                for (const CompNode& cn : comp) mw = std::max(mw, cn.wt);
                std::fprintf(stderr, "trace d=%2d c=%2zu nodes=%5zu comp=%5zu max_m=%4d max_wt=%5d max_k=%4d  A=%8.2f ms  B=%8.2f ms",
                             d, c, nodes.size(), comp.size(), mm, mw, mk, tc1 - tc0, now_ms() - tc1);
                long long ph[7] = {0, 0, 0, 0, 0, 0, 0};
                long long tp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (size_t q2 = 0; q2 < stamps.size() / 16; ++q2) {
                    for (int k = 0; k < 7; ++k)
                        ph[k] = std::max(ph[k], stamps[16 * q2 + k + 1] - stamps[16 * q2 + k]);
                    for (int k = 0; k < 8; ++k) tp[k] = std::max(tp[k], stamps[16 * q2 + 8 + k]);
                }
                std::fprintf(stderr, "  kcycles load %lld tri0 %lld gcref %lld tri %lld lmax %lld count %lld"
                             " | tri: col %lld refl %lld symv %lld t12 %lld comb %lld red %lld wb %lld trail %lld\n",
                             ph[0] / 1000, ph[1] / 1000, ph[2] / 1000, ph[3] / 1000, ph[4] / 1000, ph[5] / 1000,
                             tp[0] / 1000, tp[1] / 1000, tp[6] / 1000, tp[2] / 1000, tp[7] / 1000, tp[3] / 1000,
                             tp[4] / 1000, tp[5] / 1000);
            }
        }
        // end of level: surface pivot failures of the last colour
        if (!dry) {
            HS_HIP(hipMemcpyAsync(h_flags, d_fail, sizeof(int) * nd, hipMemcpyDeviceToHost, st));
            HS_HIP(hipStreamSynchronize(st));
            for (int s = 0; s < nd; ++s)
                if (h_flags[s]) {
                    P.stats.fail_level = d;
                    P.stats.fail_node = s;
                    throw Error{HSOLVE_ERR_NOT_SPD, "pivot block not positive definite"};
                }
        }
        P.stage.reset();
    }
    if constexpr (F32) {
        // the FP32 factor is what the single-precision solve phase reads
        for (int d = 0; d < nlev; ++d)
            for (NodeNum& nn : P.num[d].node) nn.Gm32 = reinterpret_cast<float*>(nn.Gm);
    } else if (P.apply32) {
        // single-precision copies of the solve-phase blocks, rounded once from the FP64 factor
        std::vector<DemoteTask> dt;
        double elems = 0.0;
        for (int d = 0; d < nlev; ++d)
            for (NodeNum& nn : P.num[d].node) {
                nn.Gm32 = nullptr;
                if (!nn.Gm || nn.m == 0) continue;
                const long long cnt = (long long)nn.ldG * nn.m;
                nn.Gm32 = P.fpool.alloc_n<float>(size_t(cnt));
                dt.push_back(DemoteTask{static_cast<const double*>(nn.Gm), nn.Gm32, cnt});
                elems += double(cnt);
            }
        for (size_t i = 0; i < dt.size(); i += 65535) {
            const int cnt = int(std::min<size_t>(65535, dt.size() - i));
            std::vector<DemoteTask> part(dt.begin() + i, dt.begin() + i + cnt);
            const DemoteTask* d_part = P.stage.upload_vec(part, P.spool, st);
            if (!dry) launch_demote(d_part, cnt, elems * cnt / dt.size(), st);
        }
        if (!dry) HS_HIP(hipStreamSynchronize(st));
        P.stage.reset();
    }
    build_apply_schedule(P);
    if (dry) return;
    HS_HIP(hipStreamSynchronize(st));
    P.factored = true;
    P.stats.factor_flops = flops;
    P.stats.max_rank = max_rank;
    P.stats.levels = L;
    P.stats.colours = P.total_colours;
    P.stats.factor_bytes = int64_t(P.fpool.high_water());
    P.stats.fail_level = -1;
    P.stats.fail_node = -1;
    P.stats.t_factor = std::chrono::duration<double>(clk::now() - t0).count();
}

void factor(Plan& P, const double* values) {
    if (P.f32) factor_t<float>(P, values);
    else factor_t<double>(P, values);
}

// Arena bound (hsolve_analyze): replay the factorization on the host with every rank at its
// largest possible value, min(m, 2p + |W|), and every merged super node capped at max_super.
// Each allocation of a real factorization is then no larger than its counterpart in the
// replay (the sequence of allocations depends only on the symbolic schedule, their sizes grow
// with m, k and |W|), so the replay's high-water marks bound the regions of any factorization
// that succeeds. The solve phase reuses the transient regions, or needs max_nrhs columns.
void size_arena(Plan& P) {
    const size_t inf = size_t(1) << 60;
    const int n = P.n;
    P.pattern_bytes = align256(sizeof(int64_t) * (size_t(n) + 1)) + align256(sizeof(int32_t) * std::max<size_t>(1, P.nnz)) +
                      align256(sizeof(double) * std::max<size_t>(1, P.nnz)) + align256(sizeof(int32_t) * 3 * size_t(n));
    P.fpool.init(nullptr, inf, "factor data");
    P.lpool[0].init(nullptr, inf, "live blocks (even depths)");
    P.lpool[1].init(nullptr, inf, "live blocks (odd depths)");
    P.spool.init(nullptr, inf, "per-colour scratch");
    P.dry = true;
    struct Back {
        Plan& P;
        ~Back() {
            P.dry = false;
            P.stage.dry = false;
            P.num.clear();
            P.sched.clear();
            P.factored = false;
        }
    } back{P};
    factor(P, nullptr);
    P.cap_live[0] = P.lpool[0].high_water();
    P.cap_live[1] = P.lpool[1].high_water();
    P.cap_scratch = P.spool.high_water();
    P.bound_factor = P.fpool.high_water();
    const int nr = std::max(1, P.opt.max_nrhs);
    const size_t ws = std::max(solve_ws_bytes(P, nr, P.opt.krylov), solve_ws_bytes(P, nr, -1));
    const size_t trans = P.cap_live[0] + P.cap_live[1] + P.cap_scratch;
    P.arena_bound = P.pattern_bytes + P.bound_factor + std::max(trans, ws);
    P.vlen = 0;
}

}  // namespace hs
