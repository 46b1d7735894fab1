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
#include <map>

#include "hs_internal.h"

namespace hs {

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
    double bytes = 0.0;
    P.sched.assign(nlev, {});
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
                    e.second.push_back(FwdContrib{nn.Gm + nn.m + nn.noff[t], src, nn.ldG, nn.m});
                }
                if (nn.k) {
                    const int64_t dst = LN.red_off[s];
                    auto& e = tg[dst];
                    e.first = FwdTarget{dst, nn.k, +1, 0, 0};
                    e.second.push_back(FwdContrib{nn.Gm + nn.m + nn.ntot, src, nn.ldG, nn.m});
                }
                BwdNode b{nn.Gm, src, nn.ldG, nn.m, nn.m + nn.ntot + nn.k, int(bs.size()), 0, 0};
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
                bytes += 8.0 * (double(nn.ntot + nn.k) * nn.m + double(nn.ldG) * nn.m);
                bytes += 8.0 * 2.0 * (2.0 * nn.m + 2.0 * nn.ntot + 2.0 * nn.k);
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
                cs.fwd_bytes += 8.0 * (double(nn.ntot + nn.k) * nn.m + nn.m + 2.0 * (nn.ntot + nn.k));
                cs.bwd_bytes += 8.0 * (double(nn.ldG) * nn.m + nn.ldG + nn.m);
            }
            cs.nfwd = int(ft.size());
            cs.max_len = max_len;
            cs.fwd_t = P.stage.upload_vec(ft, P.apool, st);
            cs.fwd_c = P.stage.upload_vec(fc, P.apool, st);
            cs.nbwd = int(bn.size());
            for (const BwdNode& b : bn) cs.max_m = std::max(cs.max_m, b.m);
            cs.bwd_n = P.stage.upload_vec(bn, P.apool, st);
            cs.bwd_s = P.stage.upload_vec(bs, P.apool, st);
            if (max_rows > 6144)
                throw Error{HSOLVE_ERR_INVALID, "super node with too many neighbour rows for the solve kernel"};
        }
    }
    P.stats.apply_bytes = bytes + 16.0 * P.n;
    HS_HIP(hipStreamSynchronize(st));
    P.stage.reset();
    P.d_scalars = P.apool.alloc_n<double>(2 + 2 * 512 + 16);
}

static void ensure_V(Plan& P, int nrhs) {
    if (P.d_V && P.V_cols >= nrhs) return;
    P.d_V = P.apool.alloc_n<double>(size_t(P.vlen) * nrhs);
    P.d_X = P.apool.alloc_n<double>(size_t(P.vlen) * nrhs);
    P.V_cols = nrhs;
}

// z = A_H^{-1} r for nrhs columns (device pointers, original unknown order)
void apply(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz) {
    if (!P.factored) throw Error{HSOLVE_ERR_STATE, "apply before factor"};
    hipStream_t st = P.stream;
    ensure_V(P, nrhs);
    const int L = P.L, nlev = std::max(L, 1);
    const int64_t ldv = P.vlen;
    for (int c = 0; c < nrhs; ++c)
        launch_fill(P.d_V + size_t(c) * ldv + P.n, 0.0, P.vlen - P.n, st);
    launch_gather_perm(r, ldr, P.d_V, ldv, P.d_perm, P.n, nrhs, st);
    for (int d = nlev - 1; d >= 0; --d)
        for (size_t c = 0; c < P.sched[d].size(); ++c) {
            const Plan::ColourSched& cs = P.sched[d][c];
            launch_fwd(cs.fwd_t, cs.fwd_c, cs.nfwd, cs.max_len, P.d_V, ldv, nrhs, cs.fwd_bytes * nrhs, st);
        }
    for (int d = 0; d < nlev; ++d)
        for (size_t c = P.sched[d].size(); c-- > 0;) {
            const Plan::ColourSched& cs = P.sched[d][c];
            launch_bwd(cs.bwd_n, cs.bwd_s, cs.nbwd, cs.max_m, P.d_V, P.d_X, ldv, nrhs, cs.bwd_bytes * nrhs,
                       st);
        }
    launch_scatter_perm(P.d_X, ldv, z, ldz, P.d_perm, P.n, nrhs, st);
}

void spmv(Plan& P, const double* x, double* y) {
    launch_spmv(P.d_row_ptr, P.d_col_idx, P.d_values, x, y, P.n, P.nnz, P.stream);
}

// PCG (Hestenes-Stiefel) with x0 = 0 on nrhs columns at once, each with its own scalars: a
// column stops changing once ||r_k|| <= tol ||b|| (by the recursion). One SpMV, one apply and
// one scalar read-back per iteration for the whole block. its[c] and rel[c] receive the
// iteration count and the final recursive relative residual of column c.
void pcg(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
         int* its, double* rel) {
    hipStream_t st = P.stream;
    const int n = P.n;
    const int64_t ld = n;
    if (!P.d_krylov || P.krylov_cols < nrhs) {
        P.d_krylov = P.apool.alloc_n<double>(size_t(n) * 5 * nrhs);
        P.d_kscal = P.apool.alloc_n<double>(size_t(nrhs) * (6 + DOTM_BLOCKS));
        P.d_kflag = P.apool.alloc_n<int>(size_t(nrhs));
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
        apply(P, nrhs, R, n, Z, n);
        launch_dots(R, Z, ld, n, nrhs, part, rzn, st);
        launch_xpby_multi(Pv, Z, ld, n, nrhs, rzn, rz, active, st);
        launch_copy_scalars(rz, rzn, nrhs, st);
    }
    copy_out();
}

}  // namespace hs
