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

// PCG (Hestenes-Stiefel) with x0 = 0 for one column. Returns the iteration count and the
// relative residual ||r_k|| / ||b|| of the recursion at exit in *rel_out; the loop stops
// when that value is <= tol.
int pcg(Plan& P, const double* b, double* x, double tol, int max_iter, double* rel_out) {
    hipStream_t st = P.stream;
    const int n = P.n;
    if (!P.d_krylov || P.krylov_cols < 4) {
        P.d_krylov = P.apool.alloc_n<double>(size_t(n) * 4);
        P.krylov_cols = 4;
    }
    if (!P.h_scalars)
        HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_scalars), 64 * sizeof(double),
                             hipHostMallocDefault));
    double* r = P.d_krylov;
    double* z = r + n;
    double* pv = z + n;
    double* q = pv + n;
    double* sc = P.d_scalars;                    // [0..1] dot results, [2..] partial sums
    double* keep = P.d_scalars + 2 + 2 * 512;    // [rz, pq, rz_new, rz_old]
    double* h = P.h_scalars;
    auto dcopy1 = [&](double* dst, const double* src) {
        HS_HIP(hipMemcpyAsync(dst, src, sizeof(double), hipMemcpyDeviceToDevice, st));
    };
    HS_HIP(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    launch_fill(x, 0.0, n, st);
    launch_dot2(b, b, nullptr, nullptr, n, sc, st);
    HS_HIP(hipMemcpyAsync(h, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    HS_HIP(hipStreamSynchronize(st));
    const double nb = std::sqrt(h[0]);
    if (nb == 0.0) {
        *rel_out = 0.0;
        return 0;
    }
    apply(P, 1, r, n, z, n);
    HS_HIP(hipMemcpyAsync(pv, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    launch_dot2(r, z, nullptr, nullptr, n, sc, st);
    dcopy1(keep, sc);                                       // rz
    int it = 0;
    double rel = 1.0;
    while (it < max_iter) {
        spmv(P, pv, q);
        launch_dot2(pv, q, nullptr, nullptr, n, sc, st);
        dcopy1(keep + 1, sc);                               // pq
        launch_axpy2(x, pv, r, q, keep, n, st);             // alpha = rz / pq
        ++it;
        launch_dot2(r, r, nullptr, nullptr, n, sc, st);
        HS_HIP(hipMemcpyAsync(h, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        HS_HIP(hipStreamSynchronize(st));
        rel = std::sqrt(h[0]) / nb;
        if (!(rel > tol)) break;
        apply(P, 1, r, n, z, n);
        launch_dot2(r, z, nullptr, nullptr, n, sc, st);
        dcopy1(keep + 2, sc);                               // rz_new
        dcopy1(keep + 3, keep);                             // rz
        launch_xpby(pv, z, keep + 2, n, st);                // p = z + (rz_new / rz) p
        dcopy1(keep, keep + 2);
    }
    *rel_out = rel;
    return it;
}

}  // namespace hs
