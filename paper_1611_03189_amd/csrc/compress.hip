// Compression of the well-separated block of one super node (§3.2 eq. local_compression /
// compression_sw; §6 eq. compression_xy / preserve), one workgroup per node.
//
// Input: the Gram matrix G = A_sw A_sw^T (m x m). Its eigenvectors are the left singular
// vectors of A_sw and its eigenvalues their squares, so "sigma_j > eps sigma_1" becomes
// "lambda_j > eps^2 lambda_max".
//   LoRaSp: U = eigenvectors of G with lambda > eps^2 lambda_max.
//   GC:     U1 = orthonormal basis of [phi_s, A_sw phi_w] (modified Gram-Schmidt, twice);
//           Householder reflectors W with W U1 = [R; 0] give the complement of U1; U2 =
//           eigenvectors of the projected Gram matrix (W G W^T)(q:, q:) with
//           lambda > eps^2 lambda_max(G), mapped back by W^T; U = [U1, U2].
// Eigen-solver, three kernels per batch of nodes:
//   k_comp_reduce  (one workgroup per node: 256 threads when the matrix sits in LDS, 512
//                  when it stays in global memory) scale G by its largest entry (decisions are
//                  relative); GC basis and projection; Householder tridiagonalisation of the
//                  projected matrix (unblocked, the matrix in registers, when m <= CMP_LDS_MAX;
//                  for larger m blocked by panels of TRI_NB reflectors until the trailing
//                  matrix fits the register form). lambda_max(G): for GC with at
//                  most four kept vectors by multisection on the tridiagonal form bordered
//                  by the kept directions, which is similar to G; otherwise G itself is
//                  tridiagonalised first. Number k2 of kept eigenvalues by a Sturm count;
//   k_comp_bisect  (1 to 64 lanes per kept eigenvalue) multisection until the bracket stops
//                  shrinking in floating point;
//   k_comp_vectors (one lane per kept eigenvalue) / k_comp_vectors_wave (one wave each)
//                  inverse iteration (also for up to RITZ_EXTRA eigenvalues past the
//                  threshold, for the refinement of the kept subspace's last directions);
//   k_comp_orth    the vectors of each cluster of eigenvalues closer than 1e-7 ||T|| made
//                  orthonormal (they span the cluster's invariant subspace);
//   k_comp_wy      block reflector factors T of the tridiagonalisation (compact WY form);
//   k_comp_bt      back-transformation of BT_COLS eigenvectors per workgroup, in LDS, by
//                  blocks of reflectors, then the GC reflectors.
#include <cfloat>
#include <type_traits>

#include "hs_device.h"

namespace hs {

constexpr int CMP_LDS_MAX = 128;
constexpr int CMP_MAX = 512;            // largest super node the compression accepts

// Per-node global work layout (doubles): reflectors H (m x m, ld m) | d, e, tau, lam (4m) |
// GC reflectors (16 m) + their tau (16) | info (8) | block reflector factors T (WY_NB x WY_NB
// per block of WY_NB tridiagonalisation reflectors) | inverse-iteration vectors and factors
// (4 m doubles per eigenvalue slot, slots padded to a multiple of 64, lane-interleaved).
// Size: cmp_work_doubles(m).
constexpr int WY_NB = CMP_WY_NB;
struct CmpWork {
    HS_G double *H, *d, *e, *tau, *lam, *gcv, *gct, *info, *wyT, *vs;
    __device__ CmpWork(double* wg, int m) {
        HS_G double* w = gp(wg);
        H = w;
        d = w + size_t(m) * m;
        e = d + m;
        tau = e + m;
        lam = tau + m;
        gcv = lam + m;
        gct = gcv + size_t(16) * m;
        info = gct + 16;
        wyT = info + 8;
        vs = wyT + size_t(CMP_WY_NB) * CMP_WY_NB * ((m + CMP_WY_NB - 1) / CMP_WY_NB);
    }
};
enum { INF_Q, INF_K2, INF_NN, INF_TNORM, INF_PIVMIN, INF_LO, INF_HI, INF_DONE };

// threads of the compression workgroup for matrices in global memory (8 waves: more loads
// in flight in the matrix-vector products and two trailing-update tiles at a time)
constexpr int CMP_GLOBAL_NT = 512;

template <int MAXN, int NTH = NT>
struct CmpShared {
    static constexpr int nth = NTH;    // threads of the workgroup that shares it
    double d[MAXN], e[MAXN], tau[MAXN], v[MAXN], w[MAXN];
    double tt[32];
    double bord[4][MAXN];      // GC border rows C (q <= 4) of the bordered tridiagonal
    double dq[16];             // its leading q x q block D
    double red[NTH / WAVE];
    double redp[2][5 * (NTH / WAVE)];    // double-buffered sums of the blocked reduction
    double scal[4];
    int iscal[4];
    int pts[NTH + 1];
};

// sum_l A(0, l) x[l] for the row starting at A (column stride ld), eight loads in flight
template <class PA, class PX>
__device__ inline double dot_rows(PA A, int ld, PX x, int len) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int l = 0;
    for (; l + 8 <= len; l += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += A[size_t(l + u) * ld] * x[l + u];
    }
    for (; l < len; ++l) a[0] += A[size_t(l) * ld] * x[l];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// A(0, l) -= vi w[l] + wi v[l] along one row (column stride ld)
template <class PA, class PV, class PW>
__device__ inline void rank2_row(PA A, int ld, double vi, double wi, PV v, PW w, int len) {
    int l = 0;
    for (; l + 8 <= len; l += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = A[size_t(l + u) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) A[size_t(l + u) * ld] = t[u] - (vi * w[l + u] + wi * v[l + u]);
    }
    for (; l < len; ++l) A[size_t(l) * ld] -= vi * w[l] + wi * v[l];
}

// Block-wide sums of v[0..nv) (nv <= 5) with one barrier: the partial sums alternate between
// two buffers, and a buffer is written again only after a later barrier.
template <class SH>
__device__ inline void block_sums_1b(double* v, int nv, SH& S, int& parity) {
    constexpr int NTH = SH::nth;
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    double* red = S.redp[parity];
    parity ^= 1;
#pragma unroll
    for (int r = 0; r < 5; ++r)
        if (r < nv) v[r] = wave_sum(v[r]);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < 5; ++r)
            if (r < nv) red[r * (NTH / WAVE) + w] = v[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        if (r < nv) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < NTH / WAVE; ++i) t += red[r * (NTH / WAVE) + i];
            v[r] = t;
        }
    }
}

// Householder tridiagonalisation of a symmetric matrix (column-major, ld), unblocked, for the
// trailing part T = H(j0.., j0..) of an nn x nn matrix, n = nn - j0 <= NG RB = 16 CB:
// reflector j acts on rows j+1.., its vector (first entry 1, implicit) is kept in H(j+2.., j)
// with tau[j]; diagonal -> d, sub-diagonal -> e (e[nn-1] = 0). With nbr > 0, the nbr border
// rows in LDS (Bl[r bst + l] = entry (r, l), l < nn) are multiplied on the right by every
// reflector, so [D, B; B^T, H] stays similar to the bordered result.
// Thread (row group rg, column block cb) keeps T(RB rg + a, CB cb + b) in registers for the
// whole reduction; the 16 column blocks of a row group are the 16 lanes of one DPP row, so a
// row of T v is summed in four DPP steps. Per reflector: its column is staged in LDS (colb,
// two buffers by the parity of the column: the update phase still reads one while the next
// column is written to the other) and every wave forms the reflector from it (the same
// arithmetic in each); the products p = tau T v go to LDS (pbuf) for the column side of the
// rank-2 update, with p^T v (and the border rows' products with v) in one block reduction.
// Two barriers per reflector. LDS scratch: 3 NG RB doubles.
template <int RB, int CB, class SH, class PH>
__device__ void tridiag_regs(PH H, int ld, int j0, int nn, SH& S, double* Bl, int bst, int nbr, double* scratch) {
    constexpr int NTH = SH::nth, NG = NTH / 16, RTN = NG * RB;
    static_assert(RTN == 16 * CB, "the register tiles cover a square");
    const int tid = threadIdx.x, lane = tid % WAVE, wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int cb = lane % 16, rg = wv * (WAVE / 16) + lane / 16;
    const int r0 = RB * rg, c0 = CB * cb;
    const int n = nn - j0;
    if (n <= 0) return;
    PH T = H + j0 + size_t(j0) * ld;
    double A[RB][CB];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b)
            A[a][b] = (r0 + a < n && c0 + b < n) ? T[(r0 + a) + size_t(c0 + b) * ld] : 0.0;
    int parity = 0;
    // rows of this wave: once all of them precede the reflector, its products and updates are
    // exact zeros and the wave skips them
    const int wave_last_row = RB * (wv + 1) * (WAVE / 16) - 1;
    constexpr int XL = (RTN + WAVE - 1) / WAVE, BL = (RTN + NTH - 1) / NTH;
    // All LDS reads below are unconditional (indexes stay inside the buffers) and the
    // conditions select among loaded values, so that the reads of a step issue together.
    for (int jl = 0; jl + 2 < n; ++jl) {
        const int j = j0 + jl;
        double* colb = scratch + (jl & 1) * RTN;
        double* pbuf = scratch + 2 * RTN;
        // column jl (all rows; zeros past n) into LDS by its column block
        if (cb == jl / CB) {
            const int bs = jl % CB;
#pragma unroll
            for (int b = 0; b < CB; ++b)
                if (b == bs) {
#pragma unroll
                    for (int a = 0; a < RB; ++a) colb[r0 + a] = A[a][b];
                }
        }
        __syncthreads();
        double xs = 0.0;
#pragma unroll
        for (int u = 0; u < XL; ++u) {
            const int r = jl + 2 + lane + u * WAVE;
            const double x = colb[min(r, RTN - 1)];
            xs += (r < n) ? x * x : 0.0;
        }
        const double xn2 = wave_sum(xs);
        const double alpha = colb[jl + 1], dj = colb[jl];
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (tid == 0) {
            S.d[j] = dj;
            S.e[j] = beta;
            S.tau[j] = tau;
        }
        for (int r = jl + 2 + tid; r < n; r += NTH) T[r + size_t(jl) * ld] = colb[r] * scal;
        if (tau == 0.0) continue;             // uniform: no barrier is skipped by part of the group
        // reflector entries of this thread's rows and columns (v(jl+1) = 1, zero above)
        double vr[RB], vc[CB], xr[RB], xc[CB];
#pragma unroll
        for (int a = 0; a < RB; ++a) xr[a] = colb[r0 + a];
#pragma unroll
        for (int b = 0; b < CB; ++b) xc[b] = colb[c0 + b];
#pragma unroll
        for (int a = 0; a < RB; ++a) vr[a] = (r0 + a == jl + 1) ? 1.0 : (r0 + a > jl + 1 ? xr[a] * scal : 0.0);
#pragma unroll
        for (int b = 0; b < CB; ++b) vc[b] = (c0 + b == jl + 1) ? 1.0 : (c0 + b > jl + 1 ? xc[b] * scal : 0.0);
        // (with one wave per SIMD the last wave sets the pace: skipping gains nothing there)
        const bool active = NTH <= 256 || wave_last_row > jl;
        double p[RB];
#pragma unroll
        for (int a = 0; a < RB; ++a) p[a] = 0.0;
        if (active) {
#pragma unroll
            for (int b = 0; b < CB; ++b)
#pragma unroll
                for (int a = 0; a < RB; ++a) p[a] += A[a][b] * vc[b];
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                const double y = row16_sum(p[a]) * tau;
                p[a] = (r0 + a > jl) ? y : 0.0;
            }
        }
        double pv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (cb == 0) {
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                pbuf[r0 + a] = p[a];
                pv[0] += p[a] * vr[a];
            }
        }
        // border rows: entries (r, j + 1 + l) of Bl times v(l), l over the trailing coordinates
        double vb[BL];
#pragma unroll
        for (int u = 0; u < BL; ++u) {
            const int l = jl + 1 + tid + u * NTH;
            const double x = colb[min(l, RTN - 1)];
            vb[u] = (l == jl + 1) ? 1.0 : (l < n ? x * scal : 0.0);
        }
        if (nbr > 0) {
#pragma unroll
            for (int u = 0; u < BL; ++u) {
                const int l = jl + 1 + tid + u * NTH;
                if (l < n) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (r < nbr) pv[1 + r] += Bl[r * bst + j0 + l] * vb[u];
                }
            }
        }
        block_sums_1b(pv, 1 + nbr, S, parity);
        const double K = 0.5 * tau * pv[0];
        if (active) {
            double wc[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) wc[b] = pbuf[c0 + b];
#pragma unroll
            for (int b = 0; b < CB; ++b) wc[b] -= K * vc[b];
#pragma unroll
            for (int a = 0; a < RB; ++a) {
                const double wr = p[a] - K * vr[a];
#pragma unroll
                for (int b = 0; b < CB; ++b) A[a][b] = fma(-vr[a], wc[b], fma(-wr, vc[b], A[a][b]));
            }
        }
        if (nbr > 0) {
#pragma unroll
            for (int u = 0; u < BL; ++u) {
                const int l = jl + 1 + tid + u * NTH;
                if (l < n) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (r < nbr) Bl[r * bst + j0 + l] -= tau * pv[1 + r] * vb[u];
                }
            }
        }
    }
    // the last diagonal entries and sub-diagonal entry, from their owners' registers
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
            const int r = r0 + a, c = c0 + b;
            if (r == c && r < n && r + 2 >= n) S.d[j0 + r] = A[a][b];
            if (n >= 2 && r == n - 1 && c == n - 2) S.e[j0 + n - 2] = A[a][b];
        }
    if (tid == 0) {
        if (n >= 2) S.tau[j0 + n - 2] = 0.0;
        S.e[nn - 1] = 0.0;
        S.tau[nn - 1] = 0.0;
    }
    __syncthreads();
}

// panel width of the blocked tridiagonalisation (8 measured faster than 10 and 12 with 8 waves:
// the per-column corrections with the panel shrink more than the trailing passes grow)
constexpr int TRI_NB = 8;

// Sum over the wave left in lane 63 only (the DPP steps of wave_sum without the read-back).
__device__ inline double wave_sum_last(double v) {
    v += dpp_move<DPP_QUAD_1032>(v, 0.0);
    v += dpp_move<DPP_QUAD_2301>(v, 0.0);
    v += dpp_move<DPP_ROR4>(v, 0.0);
    v += dpp_move<DPP_ROR8>(v, 0.0);
    v += dpp_move<DPP_BCAST15, 0xA>(v, 0.0);
    v += dpp_move<DPP_BCAST31, 0xC>(v, 0.0);
    return v;
}

// One wave's share of y = A v: columns [cb, ce) of the len x len matrix at A (column
// stride ld, len >= 2). Lane l takes the row pairs (r, r + 1), r = 2l + rofs + rstep k, k < KM,
// loaded as one 16-byte access; SB columns are taken at a time with every load issued before
// the products (16 / KM columns, at least 4: about 32 values per lane per round). Pairs
// that start past len - 2 are clamped to (len - 2, len - 1).
template <int KM>
__device__ inline void symv_part(const HS_G double* A, int ld, const double* v, int len, int cb, int ce,
                                 int lane, int rofs, int rstep, double* acc) {
    constexpr int SB = (16 / KM > 4) ? 16 / KM : 4;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    int rr[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) rr[k] = min(2 * lane + rofs + rstep * k, len - 2);
    for (int l0 = cb; l0 < ce; l0 += SB) {
        double a[SB][KM][2];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const HS_G double* cl = A + size_t(min(l0 + u, ce - 1)) * ld;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                a[u][k][0] = cl[rr[k]];
                a[u][k][1] = cl[rr[k] + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const double vl = (l0 + u < ce) ? v[l0 + u] : 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                acc[2 * k] += a[u][k][0] * vl;
                acc[2 * k + 1] += a[u][k][1] * vl;
            }
        }
    }
}

// Blocked form of the tridiagonalisation for matrices in global memory (same outputs): reflectors
// are generated TRI_NB columns at a time; inside a panel the trailing matrix is not
// updated, its product with each new reflector is corrected with the panel's earlier
// reflectors V and update vectors W (A_cur = A - V W^T - W V^T), and the whole trailing
// matrix takes the rank-2 nb update once per panel. LDS: Vl, Wl (TRI_NB x nn, column c
// at c nn, absolute rows) and Pp (waves x nn partial products of the matrix-vector step).
template <class SH>
__device__ void tridiagonalize_blk(HS_G double* H, int ld, int nn, SH& S, double* Bl, int bst, int nbr,
                                   double* Vl, double* Wl, double* Pp, long long* prof = nullptr) {
    constexpr int NTH = SH::nth, NW = NTH / WAVE;
    const int tid = threadIdx.x, lane = tid % WAVE, wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int nref = nn - 2;
    int parity = 0;
    long long pc[8] = {0, 0, 0, 0, 0, 0, 0, 0}, tprev = 0;   // trace: cycles per phase
    auto phase = [&](int k) {
        if (prof && tid == 0) {
            const long long t = clock64();
            if (k >= 0) pc[k] += t - tprev;
            tprev = t;
        }
    };
    phase(-1);
    // panels while the trailing matrix is larger than the register-resident form holds
    constexpr int RT_RB = 5, RT_CB = 10, RT_N = (NTH / 16) * RT_RB;
    int j0 = 0;
    for (; j0 < nref && nn - j0 > RT_N; j0 += TRI_NB) {
        const int nb = min(TRI_NB, nref - j0);
        for (int i = 0; i < nb; ++i) {
            const int j = j0 + i;
            HS_G double* col = H + size_t(j) * ld;
            // column j (rows j..), brought up to date with the panel so far, into LDS (S.w);
            // the squared norm of rows j+2.. on the way
            double* cb = S.w;
            double nrm[1] = {0.0};
            for (int r = j + tid; r < nn; r += NTH) {
                double a = col[r];
#pragma unroll
                for (int c = 0; c < TRI_NB - 1; ++c)
                    if (c < i) a -= Vl[c * nn + r] * Wl[c * nn + j] + Wl[c * nn + r] * Vl[c * nn + j];
                cb[r] = a;
                if (r == j) col[r] = a;             // diagonal entry d_j
                if (r >= j + 2) nrm[0] += a * a;
            }
            block_sums_1b(nrm, 1, S, parity);
            phase(0);
            const double xn2 = nrm[0];
            const double alpha = cb[j + 1];
            double tau = 0.0, beta = alpha, scal = 0.0;
            if (xn2 > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            // reflector: kept in H(j+2.., j) for the back-transformation and in Vl(:, i)
            for (int r = tid; r < nn; r += NTH) {
                const double vr = (r <= j) ? 0.0 : (r == j + 1 ? 1.0 : cb[r] * scal);
                Vl[i * nn + r] = vr;
                if (r >= j + 2) col[r] = vr;
            }
            if (tid == 0) {
                S.tau[j] = tau;
                S.e[j] = beta;
            }
            __syncthreads();
            phase(1);
            const int len = nn - j - 1;
            const double* v = Vl + i * nn + (j + 1);          // trailing coordinates
            double* wcol = Wl + i * nn;
            if (tau != 0.0) {
                // t1 = W(j+1:, :i)^T v, t2 = V(j+1:, :i)^T v: wave wv takes products wv, wv + 4, ..
                for (int g = wv; g < 2 * i; g += NTH / WAVE) {
                    const double* P = (g < i) ? Wl + g * nn + j + 1 : Vl + (g - i) * nn + j + 1;
                    double a = 0.0;
                    for (int r = lane; r < len; r += WAVE) a += P[r] * v[r];
                    a = wave_sum_last(a);
                    if (lane == WAVE - 1) S.tt[g] = a;
                }
                // y = A(j+1:, j+1:) v: the columns in one group per wave, each over all rows
                // (row pairs over the lanes, 128-row blocks in the same round of loads);
                // partial sums of column group g in Pp(g nn + r)
                {
                    const HS_G double* A0 = H + size_t(j + 1) * ld + (j + 1);
                    const int cw = (len + NW - 1) / NW, cbeg = wv * cw, cend = min(len, cbeg + cw);
                    const int kb = (len + 127) / 128;                // row blocks (at most 4)
                    double acc[8];
                    if (cbeg < cend) {
                        switch (kb) {
                            case 1: symv_part<1>(A0, ld, v, len, cbeg, cend, lane, 0, 128, acc); break;
                            case 2: symv_part<2>(A0, ld, v, len, cbeg, cend, lane, 0, 128, acc); break;
                            case 3: symv_part<3>(A0, ld, v, len, cbeg, cend, lane, 0, 128, acc); break;
                            default: symv_part<4>(A0, ld, v, len, cbeg, cend, lane, 0, 128, acc); break;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) acc[k] = 0.0;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int r0 = 2 * lane + 128 * k;
                        if (k < kb && r0 < len) {
                            if (r0 <= len - 2) {
                                Pp[wv * nn + r0] = acc[2 * k];
                                Pp[wv * nn + r0 + 1] = acc[2 * k + 1];
                            } else {                        // last row of an odd length
                                Pp[wv * nn + r0] = acc[2 * k + 1];
                            }
                        }
                    }
                }
                __syncthreads();
                phase(6);
                phase(2);
                double pv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
                for (int r = tid; r < len; r += NTH) {
                    double y = 0.0;
#pragma unroll
                    for (int g = 0; g < NW; ++g) y += Pp[g * nn + r];
#pragma unroll
                    for (int c = 0; c < TRI_NB - 1; ++c)
                        if (c < i) y -= Vl[c * nn + j + 1 + r] * S.tt[c] + Wl[c * nn + j + 1 + r] * S.tt[i + c];
                    const double w = tau * y;
                    S.w[r] = w;
                    pv[0] += w * v[r];
                }
                if (prof) {
                    __syncthreads();
                    phase(7);
                }
                // v^T w and the border rows' products with v, one reduction
                double* B1 = nbr ? Bl + (j + 1) : nullptr;
                for (int l = tid; l < len; l += NTH) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (r < nbr) pv[1 + r] += B1[r * bst + l] * v[l];
                }
                block_sums_1b(pv, 1 + nbr, S, parity);
                phase(3);
                const double K = 0.5 * tau * pv[0];
                for (int r = tid; r < nn; r += NTH)
                    wcol[r] = (r <= j) ? 0.0 : S.w[r - j - 1] - K * v[r - j - 1];
                for (int l = tid; l < len; l += NTH) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (r < nbr) B1[r * bst + l] -= tau * pv[1 + r] * v[l];
                }
            } else {
                for (int r = tid; r < nn; r += NTH) wcol[r] = 0.0;
            }
            __syncthreads();
            phase(4);
        }
        // trailing matrix (rows and columns from t0 on) -= V W^T + W V^T on the FP64 matrix
        // cores: 64 x 64 tiles, taken by groups of 4 waves (NG groups, tiles g, g + NG, ..);
        // wave wq of a group takes the 32 x 32 quarter (rows 32 (wq % 2), columns 32 (wq / 2))
        // as 2 x 2 blocks of v_mfma_f64_16x16x4f64 with K = 2 nb (V and W side by side, padded
        // to a multiple of 4). The product is formed transposed (operand A runs
        // over the tile's columns, operand B over its rows), so that lane l's accumulator
        // register t is C(l % 16, l / 16 + 4 t) of its block: 16 consecutive rows per column.
        // The next tile's entries are loaded before the current tile is multiplied; rows and
        // columns past nn are read clamped and never stored.
        {
            constexpr int NG = NTH / WAVE / 4;
            const int t0 = j0 + nb, tn = nn - t0, Tb = (tn + 63) / 64;
            const int tg = wv / 4, wq = wv % 4;
            const int qr = 32 * (wq % 2), qc = 32 * (wq / 2);
            const int li = lane % 16, lk = lane / 16;
            int rr[2], cc[2][4];
            dbl4 nxt[2][2];
            auto tile_pos = [&](int bt) {
                const int rb = t0 + 64 * (bt % Tb) + qr, sb = t0 + 64 * (bt / Tb) + qc;
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) rr[bi] = rb + 16 * bi + li;
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int t = 0; t < 4; ++t) cc[bj][t] = sb + 16 * bj + lk + 4 * t;
            };
            auto load_tile = [&]() {
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            nxt[bi][bj][t] = H[min(rr[bi], nn - 1) + size_t(min(cc[bj][t], nn - 1)) * ld];
            };
            if (tg < Tb * Tb) {
                tile_pos(tg);
                load_tile();
            }
            for (int bt = tg; bt < Tb * Tb; bt += NG) {
                dbl4 acc[2][2];
                int r_cur[2], c_cur[2][4];
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) {
                    r_cur[bi] = rr[bi];
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = nxt[bi][bj];
                }
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int t = 0; t < 4; ++t) c_cur[bj][t] = cc[bj][t];
                // operand columns and rows of this lane: s (tile column) for A, r (tile row) for B
                int sa[2], rbq[2];
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) sa[bj] = min(c_cur[bj][0] - lk + li, nn - 1);
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) rbq[bi] = min(r_cur[bi], nn - 1);
                if (bt + NG < Tb * Tb) {
                    tile_pos(bt + NG);
                    load_tile();
                }
                // all 2 TRI_NB / 4 steps, unrolled (operands past 2 nb are zero: the products
                // add exact zeros), so that the operand reads of a tile issue together
#pragma unroll
                for (int ks = 0; ks < 2 * TRI_NB / 4; ++ks) {
                    const int kk = 4 * ks + lk;           // this lane's K index
                    const bool kv = kk < 2 * nb;
                    const int c = kv ? (kk < nb ? kk : kk - nb) : 0;
                    const double* Ps = (kk < nb) ? Wl : Vl;   // B panel: [W, V] over tile columns
                    const double* Pr = (kk < nb) ? Vl : Wl;   // A panel: [V, W] over tile rows
                    double a[2], b[2];
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj) a[bj] = kv ? -Ps[c * nn + sa[bj]] : 0.0;
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi) b[bi] = kv ? Pr[c * nn + rbq[bi]] : 0.0;
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj)
                            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bj], b[bi], acc[bi][bj], 0, 0, 0);
                }
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            if (r_cur[bi] < nn && c_cur[bj][t] < nn)
                                H[r_cur[bi] + size_t(c_cur[bj][t]) * ld] = acc[bi][bj][t];
            }
        }
        __syncthreads();
        phase(5);
    }
    if (prof && tid == 0)
        for (int k = 0; k < 8; ++k) prof[k] = pc[k];
    for (int j = tid; j < j0; j += NTH) S.d[j] = H[j + size_t(j) * ld];
    // the rest in registers (the panel buffers are free now)
    tridiag_regs<RT_RB, RT_CB>(H, ld, j0, nn, S, Bl, bst, nbr, Vl);
}

// number of eigenvalues of the tridiagonal (d, e) below x
__device__ int sturm_count(const double* d, const double* e, int nn, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < nn; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Gershgorin interval, pivmin and norm of (S.d, S.e) into S.scal[0..3]
template <class SH>
__device__ void tridiag_bounds(int nn, SH& S) {
    if (threadIdx.x == 0) {
        double lo = S.d[0], hi = S.d[0], me = 0.0, tn = 0.0;
        for (int i = 0; i < nn; ++i) {
            const double r = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i + 1 < nn ? fabs(S.e[i]) : 0.0);
            lo = fmin(lo, S.d[i] - r);
            hi = fmax(hi, S.d[i] + r);
            if (i + 1 < nn) me = fmax(me, S.e[i] * S.e[i]);
            tn = fmax(tn, fabs(S.d[i]) + fabs(S.e[i]));
        }
        const double pad = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 1e-300;
        S.scal[0] = lo - pad;
        S.scal[1] = hi + pad;
        S.scal[2] = fmax(1e-300, 1e-300 * me);
        S.scal[3] = tn;
    }
    __syncthreads();
}

// Rounds of the 257-point multisections for lambda_max. It only sets the threshold
// eps^2 lambda_max of the kept count, so 5 rounds suffice: the bracket is 257^-5 < 2^-40 of
// its start interval (at most ||G||_F <= sqrt(m) lambda_max wide), a relative error below
// 2e-11, and a rank decided closer than that to the threshold is a tie in any arithmetic.
constexpr int BL_ROUNDS = 5;

// largest eigenvalue by parallel multisection (after tridiag_bounds)
template <class SH>
__device__ double largest_eigenvalue(int nn, SH& S) {
    constexpr int NTH = SH::nth;
    const int tid = threadIdx.x;
    double lo = S.scal[0], hi = S.scal[1];
    const double pivmin = S.scal[2];
    constexpr int NP = NTH < 256 ? NTH : 256;          // points per round (threads taking part)
    for (int round = 0; round < BL_ROUNDS; ++round) {
        const double x = lo + (hi - lo) * double(tid + 1) / double(NP + 1);
        if (tid < NP) S.pts[tid] = sturm_count(S.d, S.e, nn, x, pivmin) == nn ? 1 : 0;
        __syncthreads();
        int t = 0;
        while (t < NP && !S.pts[t]) ++t;
        const double xl = (t == 0) ? lo : lo + (hi - lo) * double(t) / double(NP + 1);
        const double xh = (t == NP) ? hi : lo + (hi - lo) * double(t + 1) / double(NP + 1);
        lo = xl;
        hi = xh;
        __syncthreads();
    }
    return 0.5 * (lo + hi);
}

// Number of eigenvalues above x of K = [D, C; C^T, T] with T = tridiag(d, e) (nn) and
// q <= 4 border rows C. Sylvester's law on the block LDL^T that eliminates T first: the
// positive pivots of T - x I (Sturm recurrence, pivots below pivmin taken as -pivmin) plus
// the positive eigenvalues of the Schur complement D - x I - C (T - x I)^{-1} C^T, the
// latter counted by an LDL^T of the q x q matrix. Used only for x at or above the largest
// eigenvalue of T, where T - x I is negative definite and no cancellation occurs.
template <int MAXN>
__device__ int bordered_count_above(const double* d, const double* e, int nn,
                                    const double (*C)[MAXN], const double* D, int q, double x,
                                    double pivmin) {
    double sc[4][4], z[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        z[a] = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) sc[a][b] = (a < q && b < q) ? D[a + 4 * b] - (a == b ? x : 0.0) : 0.0;
    }
    int cnt = 0;
    double ipp = 0.0, eprev = 0.0;          // 1 / previous pivot, previous off-diagonal
    for (int i = 0; i < nn; ++i) {
        const double l = eprev * ipp;
        double p = d[i] - x - l * eprev;
        if (fabs(p) < pivmin) p = -pivmin;
        if (p > 0.0) ++cnt;
        const double ip = 1.0 / p;
#pragma unroll
        for (int a = 0; a < 4; ++a)
            if (a < q) z[a] = C[a][i] - l * z[a];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b)
                if (b < q) sc[a][b] -= z[a] * z[b] * ip;
        ipp = ip;
        eprev = e[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= q) break;
        double piv = sc[k][k];
        if (fabs(piv) < pivmin) piv = -pivmin;
        if (piv > 0.0) ++cnt;
#pragma unroll
        for (int a = k + 1; a < 4; ++a)
#pragma unroll
            for (int b = a; b < 4; ++b)
                if (b < q) sc[a][b] -= sc[k][a] * sc[k][b] / piv;
    }
    return cnt;
}

// Counts of eigenvalues above x[0..NX) of the bordered matrix for a border of at most two
// rows: the same recurrences as bordered_count_above, NX interleaved so that their
// division chains overlap.
template <int NX, int MAXN>
__device__ void bordered_counts2(const double* d, const double* e, int nn, const double (*C)[MAXN],
                                 const double* D, int q, const double* x, double pivmin, int* cnt) {
    double s00[NX], s01[NX], s11[NX], z0[NX], z1[NX], ipp[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        s00[k] = (q > 0) ? D[0] - x[k] : 0.0;
        s01[k] = (q > 1) ? D[4] : 0.0;
        s11[k] = (q > 1) ? D[5] - x[k] : 0.0;
        z0[k] = z1[k] = 0.0;
        ipp[k] = 0.0;
        cnt[k] = 0;
    }
    double eprev = 0.0;
    for (int i = 0; i < nn; ++i) {
        const double di = d[i], c0 = C[0][i], c1 = C[1][i];
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            const double l = eprev * ipp[k];
            double p = di - x[k] - l * eprev;
            if (fabs(p) < pivmin) p = -pivmin;
            cnt[k] += (p > 0.0);
            const double ip = 1.0 / p;
            z0[k] = c0 - l * z0[k];
            z1[k] = c1 - l * z1[k];
            s00[k] -= z0[k] * z0[k] * ip;
            s01[k] -= z0[k] * z1[k] * ip;
            s11[k] -= z1[k] * z1[k] * ip;
            ipp[k] = ip;
        }
        eprev = e[i];
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        if (q > 0) {
            double p0 = s00[k];
            if (fabs(p0) < pivmin) p0 = -pivmin;
            cnt[k] += (p0 > 0.0);
            if (q > 1) {
                double p1 = s11[k] - s01[k] * s01[k] / p0;
                if (fabs(p1) < pivmin) p1 = -pivmin;
                cnt[k] += (p1 > 0.0);
            }
        }
    }
}

// block-wide minimum of an int
template <class SH>
__device__ inline int block_min_int(int v, SH& S) {
    constexpr int NTH = SH::nth;
    for (int o = WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, WAVE));
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) S.pts[w] = v;
    __syncthreads();
    int r = S.pts[0];
    for (int i = 1; i < NTH / WAVE; ++i) r = min(r, S.pts[i]);
    return r;
}

// largest eigenvalue of the bordered matrix by multisection of [lo, hi] (lo below it): each
// round evaluates one point per thread on up to 256 threads (more waves per SIMD would slow
// the latency-bound recurrences) and keeps the subinterval where the count above x drops to
// zero (BL_ROUNDS rounds).
template <class SH>
__device__ double bordered_largest(int nn, int q, double lo, double hi, SH& S) {
    constexpr int NTH = SH::nth;
    const int tid = threadIdx.x;
    const double pivmin = S.scal[2];
    constexpr int NPT = NTH < 256 ? NTH : 256;        // threads taking part (points per round)
    if (q <= 2) {
        // one point per thread: with one wave per SIMD the interleaved recurrences of several
        // points are bound by instruction issue, one recurrence by its latency only
        constexpr int NX = 1, NP = NX * NPT;
        for (int round = 0; round < BL_ROUNDS; ++round) {
            double x[NX];
            int cnt[NX];
#pragma unroll
            for (int k = 0; k < NX; ++k) x[k] = lo + (hi - lo) * double(NX * tid + k + 1) / double(NP + 1);
            int first = NP;                                   // first point with no eigenvalue above
            if (tid < NPT) {
                bordered_counts2<NX>(S.d, S.e, nn, S.bord, S.dq, q, x, pivmin, cnt);
#pragma unroll
                for (int k = NX - 1; k >= 0; --k)
                    if (cnt[k] == 0) first = NX * tid + k;
            }
            const int t = block_min_int(first, S);
            const double xl = (t == 0) ? lo : lo + (hi - lo) * double(t) / double(NP + 1);
            const double xh = (t == NP) ? hi : lo + (hi - lo) * double(t + 1) / double(NP + 1);
            lo = xl;
            hi = xh;
        }
        return 0.5 * (lo + hi);
    }
    for (int round = 0; round < BL_ROUNDS; ++round) {
        const double x = lo + (hi - lo) * double(tid + 1) / double(NPT + 1);
        const int first =
            (tid < NPT && bordered_count_above(S.d, S.e, nn, S.bord, S.dq, q, x, pivmin) == 0) ? tid : NPT;
        const int t = block_min_int(first, S);
        const double xl = (t == 0) ? lo : lo + (hi - lo) * double(t) / double(NPT + 1);
        const double xh = (t == NPT) ? hi : lo + (hi - lo) * double(t + 1) / double(NPT + 1);
        lo = xl;
        hi = xh;
    }
    return 0.5 * (lo + hi);
}


// LU factorisation with partial pivoting of the tridiagonal T - lambda I, for repeated
// solves: U has the diagonals u0 (kept as reciprocals r0), u1, u2; row i + 1 is eliminated
// with multiplier mult[i] after rows i, i + 1 were interchanged when swp[i]. Pivots smaller
// than `tiny` are raised to +-tiny (the shift may be an exact eigenvalue).
__device__ void tridiag_shift_factor(const double* d, const double* e, int nn, double lambda, double tiny,
                                     double* r0, double* u1, double* u2, double* mult, int* swp) {
    double p0 = d[0] - lambda, p1 = nn > 1 ? e[0] : 0.0, p2 = 0.0;
    for (int i = 0; i + 1 < nn; ++i) {
        const double b = e[i];
        const double a1 = d[i + 1] - lambda;
        const double c1 = (i + 2 < nn) ? e[i + 1] : 0.0;
        double np0, np1;
        if (fabs(b) > fabs(p0) && fabs(b) >= tiny) {
            const double mu = p0 / b;
            r0[i] = 1.0 / b; u1[i] = a1; u2[i] = c1;
            mult[i] = mu;
            swp[i] = 1;
            np0 = p1 - mu * a1;
            np1 = p2 - mu * c1;
        } else {
            if (fabs(p0) < tiny) p0 = (p0 < 0.0) ? -tiny : tiny;    // floor tiny pivots
            const double mu = b / p0;
            r0[i] = 1.0 / p0; u1[i] = p1; u2[i] = p2;
            mult[i] = mu;
            swp[i] = 0;
            np0 = a1 - mu * p1;
            np1 = c1 - mu * p2;
        }
        p0 = np0;
        p1 = np1;
        p2 = 0.0;
    }
    r0[nn - 1] = 1.0 / ((fabs(p0) < tiny) ? ((p0 < 0.0) ? -tiny : tiny) : p0);
}

// y <- (T - lambda I)^{-1} y with the factors of tridiag_shift_factor
__device__ void tridiag_shift_apply(int nn, const double* r0, const double* u1, const double* u2,
                                    const double* mult, const int* swp, double* y) {
    for (int i = 0; i + 1 < nn; ++i) {
        if (swp[i]) {
            const double yi = y[i];
            y[i] = y[i + 1];
            y[i + 1] = yi - mult[i] * y[i + 1];
        } else {
            y[i + 1] -= mult[i] * y[i];
        }
    }
    y[nn - 1] *= r0[nn - 1];
    if (nn >= 2) y[nn - 2] = (y[nn - 2] - u1[nn - 2] * y[nn - 1]) * r0[nn - 2];
    for (int i = nn - 3; i >= 0; --i) y[i] = (y[i] - u1[i] * y[i + 1] - u2[i] * y[i + 2]) * r0[i];
}

__device__ inline double start_value(int i, int c) {
    uint32_t h = uint32_t(i) * 2654435761u ^ (uint32_t(c) * 2246822519u + 374761393u);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    return 0.5 + double(h & 0xffffu) / 65536.0;       // in [0.5, 1.5): no zero components
}

// Two-sided application of I - tau v v^T to the symmetric m x m matrix H.
template <class SH, class PH, class PV>
__device__ void reflect_two_sided(PH H, int ld, int m, PV v, double tau, SH& S) {
    constexpr int NTH = SH::nth;
    const int tid = threadIdx.x;
    double pv_part = 0.0;
    for (int i = tid; i < m; i += NTH) {
        const double acc = tau * dot_rows(H + i, ld, v, m);
        S.w[i] = acc;
        pv_part += acc * v[i];
    }
    const double K = 0.5 * tau * block_sum<NTH>(pv_part, S.red);
    for (int i = tid; i < m; i += NTH) S.w[i] -= K * v[i];
    __syncthreads();
    for (int i = tid; i < m; i += NTH) rank2_row(H + i, ld, v[i], S.w[i], v, S.w, m);
    __syncthreads();
}


// H <- Q^T H Q for Q = H_0 H_1 .. H_{q-1}, H_t = I - tau_t v_t v_t^T (the GC reflectors, q <= 8,
// v_t at gcv + t m), in two passes over H instead of two per reflector: with the compact
// form Q = I - V T V^T (T upper triangular, T_tt = tau_t, T(0:t, t) = -tau_t T(0:t, 0:t)
// V(:, 0:t)^T v_t), Y = H V and Wm = Y T - V (T^T (V^T Y) T) / 2, the result is
// H - Wm V^T - V Wm^T. LDS (the dynamic buffer, free before the tridiagonalisation): V, Y, Wm
// (m x q each) and T, V^T V, V^T Y, T^T (V^T Y) T (q x q each).
template <class SH>
__device__ void gc_block_reflect(HS_G double* H, int ld, int m, int q, const HS_G double* gcv,
                                 const HS_G double* gct, double* buf, SH& S) {
    constexpr int NTH = SH::nth, GR = 16;
    const int tid = threadIdx.x;
    double* Vs = buf;
    double* Y = Vs + size_t(q) * m;
    double* Wm = Y + size_t(q) * m;
    double* Ts = Wm + size_t(q) * m;          // q x q, (a, b) at a + 8 b
    double* VV = Ts + 64;
    double* VY = VV + 64;
    double* Z = VY + 64;
    double* TM = Z + 64;                     // (V^T Y) T, in LDS (a private array would need scratch)
    for (int e = tid; e < q * m; e += NTH) Vs[e] = gcv[e];
    __syncthreads();
    // Y = H V: two adjacent lanes per row, each over half of the columns
    const int hm = m / 2;
    for (int tb = 0; tb < 2 * m; tb += NTH) {             // uniform trip count (the shuffle)
        const int t = tb + tid;
        const int i = min(t >> 1, m - 1), c0 = (t & 1) ? hm : 0, c1 = (t & 1) ? m : hm;
        double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (t < 2 * m) {
            // GR columns per round: their loads are in flight together (same order of sums)
            int l = c0;
            for (; l + GR <= c1; l += GR) {
                double h[GR];
#pragma unroll
                for (int u = 0; u < GR; ++u) h[u] = H[i + size_t(l + u) * ld];
#pragma unroll
                for (int u = 0; u < GR; ++u)
#pragma unroll
                    for (int b = 0; b < 8; ++b)
                        if (b < q) acc[b] += h[u] * Vs[(l + u) + b * m];
            }
            for (; l < c1; ++l) {
                const double h = H[i + size_t(l) * ld];
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    if (b < q) acc[b] += h * Vs[l + b * m];
            }
        }
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] += __shfl_xor(acc[b], 1, WAVE);
        if (t < 2 * m && !(t & 1)) {
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < q) Y[i + b * m] = acc[b];
        }
    }
    __syncthreads();
    // V^T V and V^T Y: one thread per entry (q^2 <= 64 of each)
    if (tid < 2 * q * q) {
        const int w = tid / (q * q), a = (tid % (q * q)) % q, b = (tid % (q * q)) / q;
        const double* R = w ? Y : Vs;
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += Vs[l + a * m] * R[l + b * m];
        (w ? VY : VV)[a + 8 * b] = acc;
    }
    __syncthreads();
    if (tid == 0) {                                       // T, forward (columns left to right)
        for (int b = 0; b < q; ++b) {
            const double tb = gct[b];
            for (int a = 0; a < b; ++a) {
                double acc = 0.0;
                for (int c = a; c < b; ++c) acc += Ts[a + 8 * c] * VV[c + 8 * b];
                Ts[a + 8 * b] = -tb * acc;
            }
            Ts[b + 8 * b] = tb;
            for (int a = b + 1; a < q; ++a) Ts[a + 8 * b] = 0.0;
        }
        // TM = (V^T Y) T, then Z = T^T (V^T Y) T
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                double acc = 0.0;
                for (int c = 0; c <= b; ++c) acc += VY[a + 8 * c] * Ts[c + 8 * b];
                TM[a + 8 * b] = acc;
            }
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b) {
                double acc = 0.0;
                for (int c = 0; c <= a; ++c) acc += Ts[c + 8 * a] * TM[c + 8 * b];
                Z[a + 8 * b] = acc;
            }
    }
    __syncthreads();
    for (int i = tid; i < m; i += NTH)                     // Wm = Y T - V Z / 2
        for (int b = 0; b < q; ++b) {
            double acc = 0.0;
            for (int c = 0; c <= b; ++c) acc += Y[i + c * m] * Ts[c + 8 * b];
            for (int c = 0; c < q; ++c) acc -= 0.5 * Vs[i + c * m] * Z[c + 8 * b];
            Wm[i + b * m] = acc;
        }
    __syncthreads();
    // H -= Wm V^T + V Wm^T: two adjacent lanes per row, row values in registers
    for (int t = tid; t < 2 * m; t += NTH) {
        const int i = t >> 1, c0 = (t & 1) ? hm : 0, c1 = (t & 1) ? m : hm;
        double wi[8], vi[8];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            wi[b] = (b < q) ? Wm[i + b * m] : 0.0;
            vi[b] = (b < q) ? Vs[i + b * m] : 0.0;
        }
        int l = c0;
        for (; l + GR <= c1; l += GR) {
            double h[GR];
#pragma unroll
            for (int u = 0; u < GR; ++u) h[u] = H[i + size_t(l + u) * ld];
#pragma unroll
            for (int u = 0; u < GR; ++u) {
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    if (b < q) h[u] -= wi[b] * Vs[(l + u) + b * m] + vi[b] * Wm[(l + u) + b * m];
                H[i + size_t(l + u) * ld] = h[u];
            }
        }
        for (; l < c1; ++l) {
            double h = H[i + size_t(l) * ld];
#pragma unroll
            for (int b = 0; b < 8; ++b)
                if (b < q) h -= wi[b] * Vs[l + b * m] + vi[b] * Wm[l + b * m];
            H[i + size_t(l) * ld] = h;
        }
    }
    __syncthreads();
}

// dynamic LDS of the global-matrix compression: the blocked tridiagonalisation's Vl, Wl and
// per-wave partial products, or the GC block reflection's V, Y, Wm (q <= 8) and q x q blocks
constexpr int TRI_LDS_DOUBLES = (2 * TRI_NB + CMP_GLOBAL_NT / WAVE + 1) * CMP_MAX;
static_assert(TRI_LDS_DOUBLES >= 3 * 8 * CMP_MAX + 5 * 64, "GC block reflection does not fit");

template <bool LDS, int MAXN>
__global__ __launch_bounds__(LDS ? NT : CMP_GLOBAL_NT) void k_comp_reduce(const CompressTask* tasks, int variant, double eps,
                                                    int* rank, int* extra, int kx_max) {
    constexpr int NTH = LDS ? NT : CMP_GLOBAL_NT;
    extern __shared__ double lds[];
    __shared__ CmpShared<MAXN, NTH> S;
    const CompressTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    CmpWork Wk(T.work, m);
    // in LDS a fixed odd column stride: the unrolled column offsets of the row products
    // become immediate LDS offsets (fewer address instructions), and rows stay bank-spread
    constexpr int LDL = MAXN + 1;
    const int ld = LDS ? LDL : m;
    using HPtr = typename std::conditional<LDS, double*, HS_G double*>::type;
    HPtr H;
    if constexpr (LDS) H = lds;
    else H = Wk.H;
    HS_G double* U = gp(T.U);
    const HS_G double* G = gp(T.G);
    // Householder tridiagonalisation: in registers for a matrix in LDS; blocked panels for a
    // global matrix until its trailing part fits the register form
    // inlined, so that sizes and strides stay scalar (an outlined call passes them in vector
    // registers and every branch on them becomes divergent)
    auto tri = [&](HPtr A, int n, double* Bl, int nbr) __attribute__((always_inline)) {
        if constexpr (LDS) tridiag_regs<8, 8>(A, LDL, 0, n, S, Bl, MAXN, nbr, lds + size_t(m) * LDL);
        else tridiagonalize_blk(A, ld, n, S, Bl, MAXN, nbr, lds, lds + TRI_NB * MAXN, lds + 2 * TRI_NB * MAXN,
                                T.tstamp ? T.tstamp + 8 : nullptr);
    };
    auto stamp = [&](int k) {
        if (T.tstamp && tid == 0) T.tstamp[k] = clock64();
    };
    stamp(0);
    double gm[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    {
        int e = tid;
        for (; e + 7 * NTH < m * m; e += 8 * NTH) {
#pragma unroll
            for (int u = 0; u < 8; ++u) gm[u] = fmax(gm[u], fabs(G[e + u * NTH]));
        }
        for (; e < m * m; e += NTH) gm[0] = fmax(gm[0], fabs(G[e]));
    }
    const double gmax = block_max<NTH>(fmax(fmax(fmax(gm[0], gm[1]), fmax(gm[2], gm[3])),
                                       fmax(fmax(gm[4], gm[5]), fmax(gm[6], gm[7]))), S.red);
    const double gscale = (gmax > 0.0 && isfinite(gmax)) ? 1.0 / gmax : 1.0;
    double fro = 0.0;
    copy_block<NTH>(H, ld, G, m, m, m, [&](double x, int, int) {
        const double g = x * gscale;
        fro += g * g;
        return g;
    });
    fro = sqrt(block_sum<NTH>(fro, S.red));
    stamp(1);
    // GC with at most 4 kept vectors: lambda_max(G) comes from the bordered tridiagonal form
    // of the projected matrix (one tridiagonalisation); otherwise G is tridiagonalised first.
    const bool bordered = variant == HSOLVE_GC && T.nz <= 4;
    double lam_max = 0.0;
    if (!bordered) {
        tri(H, m, nullptr, 0);
        tridiag_bounds(m, S);
        lam_max = (gmax > 0.0) ? largest_eigenvalue(m, S) : 0.0;
    }
    stamp(2);
    int q = 0;
    if (variant == HSOLVE_GC) {
        for (int c = 0; c < T.nz && q < m; ++c) {
            const HS_G double* z = gp(T.Z) + size_t(c) * m;
            HS_G double* u = U + size_t(q) * m;
            double part = 0.0;
            for (int i = tid; i < m; i += NTH) {
                u[i] = z[i];
                part += z[i] * z[i];
            }
            const double nz = sqrt(block_sum<NTH>(part, S.red));
            if (nz == 0.0) continue;
            for (int pass = 0; pass < 2; ++pass)
                for (int b = 0; b < q; ++b) {
                    const HS_G double* ub = U + size_t(b) * m;
                    double pp = 0.0;
                    for (int i = tid; i < m; i += NTH) pp += ub[i] * u[i];
                    const double dot = block_sum<NTH>(pp, S.red);
                    for (int i = tid; i < m; i += NTH) u[i] -= dot * ub[i];
                    __syncthreads();
                }
            part = 0.0;
            for (int i = tid; i < m; i += NTH) part += u[i] * u[i];
            const double nu = sqrt(block_sum<NTH>(part, S.red));
            if (nu > 1e-10 * nz) {
                for (int i = tid; i < m; i += NTH) u[i] /= nu;
                __syncthreads();
                ++q;
            }
        }
        // reflectors H_t with (H_{q-1}..H_0) U1 = [R; 0]; project G on the complement of U1
        if (!bordered)
            copy_block<NTH>(H, ld, G, m, m, m, [&](double x, int, int) { return x * gscale; });
        __syncthreads();
        double* x = S.v;        // free until the next tridiagonalisation
        for (int t = 0; t < q; ++t) {
            for (int i = tid; i < m; i += NTH) x[i] = U[i + size_t(t) * m];
            __syncthreads();
            for (int b = 0; b < t; ++b) {
                const HS_G double* vb = Wk.gcv + size_t(b) * m;
                double pp = 0.0;
                for (int i = tid; i < m; i += NTH) pp += vb[i] * x[i];
                const double dot = block_sum<NTH>(pp, S.red) * Wk.gct[b];
                for (int i = tid; i < m; i += NTH) x[i] -= dot * vb[i];
                __syncthreads();
            }
            double part = 0.0;
            for (int i = t + 1 + tid; i < m; i += NTH) part += x[i] * x[i];
            const double xn2 = block_sum<NTH>(part, S.red);
            const double alpha = x[t];
            HS_G double* vt = Wk.gcv + size_t(t) * m;
            double tau = 0.0;
            if (xn2 > 0.0) {
                const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                const double scal = 1.0 / (alpha - beta);
                for (int i = tid; i < m; i += NTH) vt[i] = (i < t) ? 0.0 : (i == t ? 1.0 : x[i] * scal);
            } else {
                for (int i = tid; i < m; i += NTH) vt[i] = (i == t) ? 1.0 : 0.0;
            }
            if (tid == 0) Wk.gct[t] = tau;
            __syncthreads();
            // in LDS one reflector at a time; a matrix in global memory takes them together below
            if (LDS || q > 8) {
                if (tau != 0.0) reflect_two_sided(H, ld, m, vt, tau, S);
            }
        }
        if constexpr (!LDS) {
            if (q > 0 && q <= 8) gc_block_reflect(H, ld, m, q, Wk.gcv, Wk.gct, lds, S);
        }
        stamp(3);
        const int nt = m - q;
        if (nt > 0) {
            if (bordered) {      // border rows move to LDS for the reduction
                for (int i = tid; i < nt; i += NTH)
                    for (int r = 0; r < q; ++r) S.bord[r][i] = H[r + size_t(q + i) * ld];
                __syncthreads();
            }
            tri(H + size_t(q) * ld + q, nt, bordered ? &S.bord[0][0] : nullptr, bordered ? q : 0);
            tridiag_bounds(nt, S);
        }
        stamp(4);
        if (bordered && gmax > 0.0) {
            // K = [D, C; C^T, T] is similar to G; lambda_max(K) >= lambda_max(T) (interlacing)
            if (tid < 16) {
                const int a = tid % 4, b = tid / 4;
                S.dq[tid] = (a < q && b < q) ? H[a + size_t(b) * ld] : 0.0;
            }
            if (nt == 0 && tid == 0) S.scal[2] = 1e-300;
            __syncthreads();
            // lower end: the largest diagonal entry of K (at most lambda_max); below the
            // largest eigenvalue of T the Sturm part of the count alone is already positive
            double dmax = -DBL_MAX;
            for (int i = tid; i < nt; i += NTH) dmax = fmax(dmax, S.d[i]);
            if (tid < q) dmax = fmax(dmax, S.dq[tid + 4 * tid]);
            dmax = block_max<NTH>(dmax, S.red);
            const double lo = dmax - 4.0 * DBL_EPSILON * fro - 1e-300;
            const double hi = fro * (1.0 + 1e-12) + 1e-300;
            lam_max = bordered_largest(nt, q, lo, hi, S);
        }
    }
    stamp(5);
    const int nn = m - q;
    const int cap = min(nn, T.wt);
    const double thr = eps * eps * fmax(lam_max, 0.0);
    if (tid == 0) {
        int k2;
        if (nn <= 0) k2 = 0;
        else if (eps == 0.0) k2 = cap;
        else k2 = min(cap, nn - sturm_count(S.d, S.e, nn, thr, S.scal[2]));
        if (k2 < 0) k2 = 0;
        if (q + k2 == 0 && cap > 0) k2 = 1;
        S.iscal[3] = k2;
    }
    __syncthreads();
    int k2 = S.iscal[3];
    if (variant == HSOLVE_LORASP && gmax == 0.0 && eps > 0.0) {
        // A_sw exactly zero: the kept direction is the first unit vector
        for (int i = tid; i < m; i += NTH) U[i] = (i == 0) ? 1.0 : 0.0;
        k2 = 0;
        q = 1;
    }
    // eigenvectors past the threshold for the Rayleigh-Ritz refinement of the last kept
    // directions (none when nothing is truncated); the later kernels compute k2 + kx vectors
    const int kx = (kx_max > 0 && eps > 0.0 && gmax > 0.0 && k2 > 0) ? max(0, min(kx_max, cap - k2)) : 0;
    for (int i = tid; i < nn; i += NTH) {
        Wk.d[i] = S.d[i];
        Wk.e[i] = S.e[i];
        Wk.tau[i] = S.tau[i];
    }
    if (LDS)
        for (int e = tid; e < m * m; e += NTH) Wk.H[e] = H[(e % m) + (e / m) * ld];
    if (tid == 0) {
        Wk.info[INF_Q] = q;
        Wk.info[INF_K2] = k2 + kx;
        Wk.info[INF_NN] = nn;
        Wk.info[INF_TNORM] = S.scal[3];
        Wk.info[INF_PIVMIN] = S.scal[2];
        Wk.info[INF_LO] = S.scal[0];
        Wk.info[INF_HI] = S.scal[1];
        rank[T.id] = q + k2;
        if (extra) extra[T.id] = kx;
    }
    stamp(6);
}

// one thread per kept eigenvalue (largest first)
// numbers of eigenvalues of the tridiagonal (d, e) below x[0..NX), NX recurrences interleaved
template <int NX>
__device__ __forceinline__ void sturm_counts(const double* d, const double* e, int nn, const double* x,
                                             double pivmin, int* cnt) {
    double q[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
        cnt[k] = 0;
        q[k] = 1.0;
    }
    double e2 = 0.0;
    for (int i = 0; i < nn; ++i) {
        const double di = d[i];
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            double t = di - x[k] - e2 / q[k];
            if (fabs(t) < pivmin) t = -pivmin;
            cnt[k] += (t < 0.0);
            q[k] = t;
        }
        e2 = e[i] * e[i];
    }
}

// Kept eigenvalues (largest first) by multisection of the Gershgorin interval: a group of LPE
// lanes per eigenvalue, each lane evaluating BIS_NX points per round (BIS_NX LPE points in
// all), until the bracket stops shrinking (adjacent floating-point numbers). Wide
// groups finish in few rounds (latency) for few nodes; narrow groups do less total work
// (throughput) when a launch holds many nodes. A lane's BIS_NX recurrences are interleaved:
// several hide the latency of one division chain when the groups are narrow, while wide
// groups take one point per lane (the lanes already give many points per round).
template <int LPE>
__global__ __launch_bounds__(NT) void k_comp_bisect(const CompressTask* tasks) {
    constexpr int BIS_NX = LPE >= 16 ? 1 : (LPE >= 4 ? 2 : 4);
    __shared__ double d[CMP_MAX], e[CMP_MAX];
    const CompressTask T = tasks[blockIdx.y];
    CmpWork Wk(T.work, T.m);
    const int k2 = int(Wk.info[INF_K2]), nn = int(Wk.info[INF_NN]);
    constexpr int GPB = NT / LPE;                  // eigenvalues per workgroup
    if (int(blockIdx.x) * GPB >= k2) return;
    for (int i = threadIdx.x; i < nn; i += NT) {
        d[i] = Wk.d[i];
        e[i] = Wk.e[i];
    }
    __syncthreads();
    const int g = threadIdx.x % LPE, j = blockIdx.x * GPB + threadIdx.x / LPE;
    if ((j - int(threadIdx.x % WAVE) / LPE) >= k2) return;      // whole wave past the last one
    const bool active = j < k2;
    const int a = nn - 1 - (active ? j : k2 - 1);                // a-th smallest
    const double pivmin = Wk.info[INF_PIVMIN];
    // Each eigenvalue is bracketed to the resolution of the floating-point Sturm count: the
    // group stops when its bracket no longer shrinks (adjacent numbers), not at an absolute
    // tolerance. The kept eigenvalues near eps^2 lambda_max are small against ||T||, and a
    // bracket of width u ||T|| would leave their last digits to the launch shape; inverse
    // iteration carries those digits into the basis. So the result does not depend on LPE.
    constexpr int NP = BIS_NX * LPE;
    double lo = Wk.info[INF_LO], hi = Wk.info[INF_HI];
    bool need = hi > lo;
    for (int round = 0; round < 64; ++round) {
        // every lane of the wave stays in the loop until all groups have converged
        int any = need ? 1 : 0;
        for (int o = WAVE / 2; o > 0; o >>= 1) any = max(any, __shfl_xor(any, o, WAVE));
        if (!any) break;
        double x[BIS_NX];
        int cnt[BIS_NX];
#pragma unroll
        for (int k = 0; k < BIS_NX; ++k) x[k] = lo + (hi - lo) * double(BIS_NX * g + k + 1) / double(NP + 1);
        sturm_counts<BIS_NX>(d, e, nn, x, pivmin, cnt);
        int first = NP;                            // first point with more than a eigenvalues below
#pragma unroll
        for (int k = BIS_NX - 1; k >= 0; --k)
            if (cnt[k] > a) first = BIS_NX * g + k;
        for (int o = LPE / 2; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, WAVE));
        const double xl = (first == 0) ? lo : lo + (hi - lo) * double(first) / double(NP + 1);
        const double xh = (first == NP) ? hi : lo + (hi - lo) * double(first + 1) / double(NP + 1);
        if (need) {
            if (xl == lo && xh == hi) need = false;       // no progress in floating point
            lo = xl;
            hi = xh;
            if (!(hi > lo)) need = false;
        }
    }
    if (active && g == 0) Wk.lam[j] = 0.5 * (lo + hi);
}

// Inverse iteration for the kept eigenvalues, one lane per eigenvalue (VL per workgroup), in
// trailing coordinates: INV_ITERS times, the LU factorisation with partial pivoting of T - lambda I
// (the steps of tridiag_shift_factor) with the forward elimination applied to y on the way,
// then the back substitution and the normalisation. Each lane keeps its vector and factors in
// the node's work buffer, lane-interleaved (row i of all lanes is one coalesced access), and
// reads eight rows ahead of its sequential recurrence.
constexpr int VL = 64;
// Passes of inverse iteration. The shifts are the eigenvalues to the last bit, so one solve
// already damps a neighbour at distance g by about ulp(lambda) / g; the second leaves it far
// below rounding.
constexpr int INV_ITERS = 2;

__global__ __launch_bounds__(VL) void k_comp_vectors(const CompressTask* tasks) {
    __shared__ double d[CMP_MAX], e[CMP_MAX];
    const CompressTask T = tasks[blockIdx.y];
    const int m = T.m;
    CmpWork Wk(T.work, m);
    const int k2 = int(Wk.info[INF_K2]), nn = int(Wk.info[INF_NN]), q = int(Wk.info[INF_Q]);
    if (int(blockIdx.x) * VL >= k2 || nn <= 0) return;
    for (int i = threadIdx.x; i < nn; i += VL) {
        d[i] = Wk.d[i];
        e[i] = Wk.e[i];
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const int c = blockIdx.x * VL + lane;
    const bool act = c < k2;
    const double lamc = Wk.lam[act ? c : k2 - 1];
    const double tnorm = Wk.info[INF_TNORM];
    const double tiny = DBL_EPSILON * (tnorm > 0.0 ? tnorm : 1.0);
    HS_G double* base = Wk.vs + size_t(blockIdx.x) * 4 * size_t(m) * VL + lane;
    auto at = [&](int f, int i) -> HS_G double& { return base[(size_t(f) * m + i) * VL]; };   // 0 y, 1 r0, 2 u1, 3 u2
    for (int i = 0; i < nn; ++i) at(0, i) = start_value(i, c);
    double inv = 1.0;
    for (int it = 0; it < INV_ITERS; ++it) {
        double p0 = d[0] - lamc, p1 = nn > 1 ? e[0] : 0.0, p2 = 0.0;
        double yc = at(0, 0) * inv;                 // current y_i after the earlier eliminations
        for (int i0 = 0; i0 + 1 < nn; i0 += 8) {
            const int nb = min(8, nn - 1 - i0);
            double ynb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < nb) ynb[u] = at(0, i0 + u + 1) * inv;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (u >= nb) break;
                const int i = i0 + u;
                const double bb = e[i], a1 = d[i + 1] - lamc, c1 = (i + 2 < nn) ? e[i + 1] : 0.0;
                const double yn = ynb[u];
                double r0, u1, u2, ys, np0, np1;
                if (fabs(bb) > fabs(p0) && fabs(bb) >= tiny) {      // rows i, i + 1 interchanged
                    const double mu = p0 / bb;
                    r0 = 1.0 / bb;
                    u1 = a1;
                    u2 = c1;
                    np0 = p1 - mu * a1;
                    np1 = p2 - mu * c1;
                    ys = yn;
                    yc = yc - mu * yn;
                } else {
                    if (fabs(p0) < tiny) p0 = (p0 < 0.0) ? -tiny : tiny;
                    const double mu = bb / p0;
                    r0 = 1.0 / p0;
                    u1 = p1;
                    u2 = p2;
                    np0 = a1 - mu * p1;
                    np1 = c1 - mu * p2;
                    ys = yc;
                    yc = yn - mu * yc;
                }
                at(1, i) = r0;
                at(2, i) = u1;
                at(3, i) = u2;
                at(0, i) = ys;
                p0 = np0;
                p1 = np1;
                p2 = 0.0;
            }
        }
        const double rl = 1.0 / ((fabs(p0) < tiny) ? ((p0 < 0.0) ? -tiny : tiny) : p0);
        // back substitution with the squared norm on the way
        double y1 = yc * rl, y2 = 0.0;
        at(0, nn - 1) = y1;
        double nrm2 = y1 * y1;
        if (nn >= 2) {
            const double y0 = (at(0, nn - 2) - at(2, nn - 2) * y1) * at(1, nn - 2);
            at(0, nn - 2) = y0;
            nrm2 += y0 * y0;
            y2 = y1;
            y1 = y0;
        }
        for (int i0 = nn - 3; i0 >= 0; i0 -= 8) {
            const int nb = min(8, i0 + 1);
            double rr[8], ua[8], ub[8], yv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < nb) {
                    rr[u] = at(1, i0 - u);
                    ua[u] = at(2, i0 - u);
                    ub[u] = at(3, i0 - u);
                    yv[u] = at(0, i0 - u);
                }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (u >= nb) break;
                const double y0 = (yv[u] - ua[u] * y1 - ub[u] * y2) * rr[u];
                at(0, i0 - u) = y0;
                nrm2 += y0 * y0;
                y2 = y1;
                y1 = y0;
            }
        }
        const double nrm = sqrt(nrm2);
        inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
    }
    if (act) {
        HS_G double* col = gp(T.U) + size_t(q + c) * m + q;
        for (int i = 0; i < nn; ++i) col[i] = at(0, i) * inv;
    }
}

// The same inverse iteration with one wave per kept eigenvalue, the factors in LDS and the
// recurrences run by lane 0: shorter latency per vector, for launches with few eigenvalues
constexpr int VNT = 128;           // two waves per workgroup in k_comp_vectors_wave

__global__ __launch_bounds__(VNT) void k_comp_vectors_wave(const CompressTask* tasks, int ldn) {
    // LDS (ldn >= every node's order): d, e, then per wave y, u0, u1, u2, mult and the
    // interchange flags
    extern __shared__ double lds[];
    double* d = lds;
    double* e = d + ldn;
    const CompressTask T = tasks[blockIdx.y];
    const int m = T.m;
    CmpWork Wk(T.work, m);
    const int k2 = int(Wk.info[INF_K2]), nn = int(Wk.info[INF_NN]), q = int(Wk.info[INF_Q]);
    if (int(blockIdx.x) * (VNT / WAVE) >= k2) return;
    for (int i = threadIdx.x; i < nn; i += VNT) {
        d[i] = Wk.d[i];
        e[i] = Wk.e[i];
    }
    __syncthreads();
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int c0 = blockIdx.x * (VNT / WAVE) + wv;
    if (c0 >= k2) return;
    const double tnorm = Wk.info[INF_TNORM];
    const HS_G double* lam = Wk.lam;
    const double tiny = DBL_EPSILON * (tnorm > 0.0 ? tnorm : 1.0);
    double* y = e + ldn + size_t(wv) * 5 * ldn;
    double* u0 = y + ldn;
    double* u1 = u0 + ldn;
    double* u2 = u1 + ldn;
    double* mult = u2 + ldn;
    int* swp = reinterpret_cast<int*>(e + ldn + size_t(VNT / WAVE) * 5 * ldn) + wv * ldn;
    const int c = c0;
    for (int i = lane; i < nn; i += WAVE) y[i] = start_value(i, c);
    wave_sync();
    if (lane == 0) tridiag_shift_factor(d, e, nn, lam[c], tiny, u0, u1, u2, mult, swp);
    for (int it = 0; it < INV_ITERS; ++it) {
        wave_sync();
        if (lane == 0) tridiag_shift_apply(nn, u0, u1, u2, mult, swp, y);
        wave_sync();
        double part = 0.0;
        for (int i = lane; i < nn; i += WAVE) part += y[i] * y[i];
        const double nrm = sqrt(wave_sum(part));
        const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
        for (int i = lane; i < nn; i += WAVE) y[i] *= inv;
    }
    HS_G double* col = gp(T.U) + size_t(q + c) * m + q;
    for (int i = lane; i < nn; i += WAVE) col[i] = y[i];
}

// Eigenvectors of a cluster (consecutive eigenvalues closer than 1e-7 ||T||) are computed
// independently from different start vectors; they span the cluster's invariant subspace
// and are made orthonormal here by modified Gram-Schmidt, twice. One wave per cluster
// leader.
__global__ __launch_bounds__(NT) void k_comp_orth(const CompressTask* tasks) {
    const CompressTask T = tasks[blockIdx.y];
    const int m = T.m;
    CmpWork Wk(T.work, m);
    const int k2 = int(Wk.info[INF_K2]), nn = int(Wk.info[INF_NN]), q = int(Wk.info[INF_Q]);
    const int lane = threadIdx.x % WAVE, c0 = blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;
    if (c0 >= k2) return;
    const double ctol = 1e-7 * Wk.info[INF_TNORM];
    const HS_G double* lam = Wk.lam;
    if (c0 > 0 && lam[c0 - 1] - lam[c0] <= ctol) return;     // not a cluster leader
    int c1 = c0 + 1;
    while (c1 < k2 && lam[c1 - 1] - lam[c1] <= ctol) ++c1;
    if (c1 - c0 < 2) return;
    HS_G double* U = gp(T.U);
    for (int c = c0; c < c1; ++c) {
        HS_G double* yc = U + size_t(q + c) * m + q;
        for (int pass = 0; pass < 2; ++pass)
            for (int b = c0; b < c; ++b) {
                const HS_G double* yb = U + size_t(q + b) * m + q;
                double part = 0.0;
                for (int i = lane; i < nn; i += WAVE) part += yb[i] * yc[i];
                const double dot = wave_sum(part);
                for (int i = lane; i < nn; i += WAVE) yc[i] -= dot * yb[i];
            }
        double part = 0.0;
        for (int i = lane; i < nn; i += WAVE) part += yc[i] * yc[i];
        const double nrm = sqrt(wave_sum(part));
        const double inv = (nrm > 0.0 && isfinite(nrm)) ? 1.0 / nrm : 0.0;
        for (int i = lane; i < nn; i += WAVE) yc[i] *= inv;
    }
}

// Block reflector factors (compact WY form): for block b of WY_NB consecutive
// tridiagonalisation reflectors, H_j0 ... H_j0+nb-1 = I - V T V^T with T upper triangular
// (T_ii = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) V(:, 0:i)^T v_i). One workgroup per block.
// Reflector j acts on the trailing coordinates: v_j(j + 1) = 1, v_j(r) = H(q + r, q + j) for
// r >= j + 2 (m-dim row q + r), zero elsewhere.
__global__ __launch_bounds__(NT) void k_comp_wy(const CompressTask* tasks) {
    __shared__ double Vs[WY_NB][CMP_MAX + 1];
    __shared__ double Gs[WY_NB][WY_NB + 1];
    __shared__ double Ts[WY_NB][WY_NB + 1];
    const CompressTask T = tasks[blockIdx.y];
    const int m = T.m;
    CmpWork Wk(T.work, m);
    const int nn = int(Wk.info[INF_NN]), q = int(Wk.info[INF_Q]), k2 = int(Wk.info[INF_K2]);
    const int nref = nn - 2;
    const int j0 = blockIdx.x * WY_NB;
    if (k2 <= 0 || j0 >= nref) return;
    const int nb = min(WY_NB, nref - j0);
    const int tid = threadIdx.x;
    for (int e = tid; e < WY_NB * nn; e += NT) {
        const int i = e / nn, r = e % nn, j = j0 + i;
        double v = 0.0;
        if (i < nb) v = (r == j + 1) ? 1.0 : (r >= j + 2 ? Wk.H[(q + r) + size_t(q + j) * m] : 0.0);
        Vs[i][r] = v;
    }
    __syncthreads();
    // Gram matrix G = V^T V (upper part), 8 lanes per entry
    for (int p = tid / 8; p < WY_NB * WY_NB; p += NT / 8) {
        const int a = p % WY_NB, c = p / WY_NB;
        double sum = 0.0;
        if (a < c && c < nb)
            for (int r = tid % 8; r < nn; r += 8) sum += Vs[a][r] * Vs[c][r];
        sum += __shfl_xor(sum, 1, WAVE);
        sum += __shfl_xor(sum, 2, WAVE);
        sum += __shfl_xor(sum, 4, WAVE);
        if (tid % 8 == 0) Gs[a][c] = sum;
    }
    __syncthreads();
    // T column by column (first wave, lane = row)
    if (tid < WAVE) {
        const int lane = tid;
        for (int i = 0; i < WY_NB; ++i)
            if (lane < WY_NB) Ts[lane][i] = 0.0;
        wave_sync();
        for (int i = 0; i < nb; ++i) {
            const double ti = Wk.tau[j0 + i];
            double t = 0.0;
            if (lane < i) {
                for (int l = lane; l < i; ++l) t += Ts[lane][l] * Gs[l][i];
                t *= -ti;
            }
            wave_sync();
            if (lane < i) Ts[lane][i] = t;
            if (lane == i) Ts[i][i] = ti;
            wave_sync();
        }
    }
    __syncthreads();
    HS_G double* Tg = Wk.wyT + size_t(blockIdx.x) * WY_NB * WY_NB;
    for (int e = tid; e < WY_NB * WY_NB; e += NT) Tg[e] = Ts[e % WY_NB][e / WY_NB];
}

// Back-transformation of the eigenvectors y (trailing coordinates, columns q.. of U) to the
// m-dim coordinates: U(:, q + c) = W_gc^T [0_q; Q y_c] with Q = B_0 ... B_{nb-1} the
// tridiagonalisation blocks (B_b = I - V_b T_b V_b^T, applied last first) and W_gc the GC
// reflectors. One workgroup per BT_COLS eigenvectors, held in LDS.
constexpr int BT_COLS = 16;
static_assert(BT_COLS == 16 && WY_NB == 16, "k_comp_bt forms 16 x 16 blocks on the matrix cores");

__global__ __launch_bounds__(NT) void k_comp_bt(const CompressTask* tasks, int variant) {
    extern __shared__ double lds[];
    const CompressTask T = tasks[blockIdx.y];
    const int m = T.m;
    CmpWork Wk(T.work, m);
    const int nn = int(Wk.info[INF_NN]), q = int(Wk.info[INF_Q]), k2 = int(Wk.info[INF_K2]);
    const int c0 = blockIdx.x * BT_COLS;
    if (c0 >= k2) return;
    const int nc = min(BT_COLS, k2 - c0);
    const int tid = threadIdx.x;
    const int ldy = m + 1;                          // Y: m x BT_COLS, column-major
    double* Y = lds;
    double* Vs = Y + size_t(BT_COLS) * ldy;        // V block: WY_NB columns of nn (ld nn + 1)
    const int ldv = nn + 1;
    double* Wm = Vs + size_t(WY_NB) * ldv;         // W = V^T Y then T W: WY_NB x BT_COLS
    double* Ts = Wm + WY_NB * BT_COLS;             // T: WY_NB x WY_NB (ld WY_NB + 1)
    double* Wp = Ts + WY_NB * (WY_NB + 1);         // partial V^T Y of the four waves
    HS_G double* U = gp(T.U);
    for (int e = tid; e < BT_COLS * m; e += NT) {
        const int c = e / m, r = e % m;
        Y[r + c * ldy] = (c < nc && r >= q) ? U[r + size_t(q + c0 + c) * m] : 0.0;
    }
    const int nref = nn - 2;
    const int nblk = nref > 0 ? (nref + WY_NB - 1) / WY_NB : 0;
    double* Yt = Y + q;                              // trailing coordinates
    for (int b = nblk - 1; b >= 0; --b) {
        const int j0 = b * WY_NB, nb = min(WY_NB, nref - j0);
        __syncthreads();
        for (int e = tid; e < WY_NB * nn; e += NT) {
            const int i = e / nn, r = e % nn, j = j0 + i;
            double v = 0.0;
            if (i < nb) v = (r == j + 1) ? 1.0 : (r >= j + 2 ? Wk.H[(q + r) + size_t(q + j) * m] : 0.0);
            Vs[r + i * ldv] = v;
        }
        const HS_G double* Tg = Wk.wyT + size_t(b) * WY_NB * WY_NB;
        for (int e = tid; e < WY_NB * WY_NB; e += NT) Ts[(e % WY_NB) + (e / WY_NB) * (WY_NB + 1)] = Tg[e];
        __syncthreads();
        // W = V^T Y on the FP64 matrix cores (16 x 16, K = the rows from j0 + 1, where V is
        // nonzero): the four waves take every fourth K step, then their partial sums are added
        {
            const int lane = tid % WAVE, wv = tid / WAVE, li = lane % 16, lk = lane / 16;
            const int r0 = j0 + 1, nks = (nn - r0 + 3) / 4;
            dbl4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int ks = wv; ks < nks; ks += NT / WAVE) {
                const int r = r0 + 4 * ks + lk;
                const bool ok = r < nn;
                const double a = ok ? Vs[r + li * ldv] : 0.0;     // A(i, r) = V(r, i)
                const double bv = ok ? Yt[r + li * ldy] : 0.0;    // B(r, c) = Y(r, c)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) Wp[wv * WY_NB * BT_COLS + (lk + 4 * t) + li * WY_NB] = acc[t];
        }
        __syncthreads();
        for (int p = tid; p < WY_NB * BT_COLS; p += NT) {
            double w = 0.0;
#pragma unroll
            for (int h = 0; h < NT / WAVE; ++h) w += Wp[h * WY_NB * BT_COLS + p];
            Wm[p] = w;
        }
        __syncthreads();
        // W <- T W (T upper triangular)
        double tw[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = tid + h * NT;
            tw[h] = 0.0;
            if (p < WY_NB * BT_COLS) {
                const int i = p % WY_NB, c = p / WY_NB;
                for (int l = i; l < WY_NB; ++l) tw[h] += Ts[i + l * (WY_NB + 1)] * Wm[l + c * WY_NB];
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = tid + h * NT;
            if (p < WY_NB * BT_COLS) Wm[p] = tw[h];
        }
        __syncthreads();
        // Y -= V W on the matrix cores, by blocks of 16 rows (wave wv takes every fourth block):
        // D(c, r) = Y(r, c) - sum_i W(i, c) V(r, i), lane l's register t is (c = l / 16 + 4 t,
        // r = l % 16 of the block)
        {
            const int lane = tid % WAVE, wv = tid / WAVE, li = lane % 16, lk = lane / 16;
            for (int rb = wv * 16; rb < nn; rb += 16 * (NT / WAVE)) {
                const int r = rb + li;
                const int rc = min(r, nn - 1);
                dbl4 acc;
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] = Yt[rc + (lk + 4 * t) * ldy];
#pragma unroll
                for (int ks = 0; ks < WY_NB / 4; ++ks) {
                    const int i = 4 * ks + lk;
                    const double a = -Wm[i + li * WY_NB];         // A(c, i) = -W(i, c)
                    const double bv = Vs[rc + i * ldv];           // B(i, r) = V(r, i)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
                }
                if (r < nn) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) Yt[r + (lk + 4 * t) * ldy] = acc[t];
                }
            }
        }
    }
    __syncthreads();
    // GC reflectors, last first: y <- (I - tau v v^T) y in m-dim coordinates
    if (variant == HSOLVE_GC) {
        double* dots = Wm;                           // BT_COLS partial sums
        for (int t = q - 1; t >= 0; --t) {
            const double tt = Wk.gct[t];
            if (tt == 0.0) continue;
            const HS_G double* vt = Wk.gcv + size_t(t) * m;
            // one wave per column: dot of v with column c
            for (int c = tid / WAVE; c < BT_COLS; c += NT / WAVE) {
                double part = 0.0;
                for (int r = tid % WAVE; r < m; r += WAVE) part += vt[r] * Y[r + c * ldy];
                part = wave_sum(part);
                if (tid % WAVE == 0) dots[c] = part * tt;
            }
            __syncthreads();
            for (int e = tid; e < m * BT_COLS; e += NT) {
                const int r = e % m, c = e / m;
                Y[r + c * ldy] -= dots[c] * vt[r];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int e = tid; e < nc * m; e += NT) {
        const int c = e / m, r = e % m;
        U[r + size_t(q + c0 + c) * m] = Y[r + c * ldy];
    }
}

// ---------------------------------------------------------------------------------
// First step of the first-order one-sided projection (Appendix B): Z = [X_s, A_sw X_w]
// (m x nz, nz <= 16) is replaced by its left singular vectors with sigma_j > eps1 sigma_1(Z)
// in its first columns and zeros after them, so that the GC basis step that follows keeps
// exactly that truncated basis. Per node: the nz x nz Gram matrix Z^T Z (one wave per pair of
// columns), its eigen-decomposition by cyclic Jacobi rotations (one lane; nz is at most 16),
// then every row of Z times V_kept / sigma_kept.
// ---------------------------------------------------------------------------------
constexpr int TRUNC_MAXZ = 16;

__global__ __launch_bounds__(NT) void k_gc_truncate(const CompressTask* tasks, double eps1) {
    const CompressTask T = tasks[blockIdx.x];
    const int m = T.m, nz = T.nz;
    if (nz <= 0 || nz > TRUNC_MAXZ) return;
    __shared__ double Gm[TRUNC_MAXZ][TRUNC_MAXZ], Vm[TRUNC_MAXZ][TRUNC_MAXZ];
    __shared__ double lam[TRUNC_MAXZ];
    __shared__ int order[TRUNC_MAXZ];
    __shared__ int nkeep;
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    HS_G double* Z = gp(const_cast<double*>(T.Z));
    const int npair = nz * (nz + 1) / 2;
    for (int pr = wv; pr < npair; pr += NT / WAVE) {
        int a = 0, r = pr;
        while (r >= nz - a) { r -= nz - a; ++a; }
        const int b = a + r;
        double part = 0.0;
        for (int i = lane; i < m; i += WAVE) part += Z[i + size_t(a) * m] * Z[i + size_t(b) * m];
        const double dot = wave_sum(part);
        if (lane == 0) { Gm[a][b] = dot; Gm[b][a] = dot; }
    }
    __syncthreads();
    if (tid == 0) {
        for (int a = 0; a < nz; ++a)
            for (int b = 0; b < nz; ++b) Vm[a][b] = (a == b) ? 1.0 : 0.0;
        double fro = 0.0;
        for (int a = 0; a < nz; ++a)
            for (int b = 0; b < nz; ++b) fro += Gm[a][b] * Gm[a][b];
        for (int sweep = 0; sweep < 60; ++sweep) {
            double off = 0.0;
            for (int a = 0; a < nz; ++a)
                for (int b = a + 1; b < nz; ++b) off += Gm[a][b] * Gm[a][b];
            if (!(off > 1e-34 * fro)) break;
            for (int a = 0; a < nz; ++a)
                for (int b = a + 1; b < nz; ++b) {
                    const double apq = Gm[a][b];
                    if (apq == 0.0) continue;
                    // rotation that zeroes (a, b): t = tan, from theta = (G_bb - G_aa) / (2 G_ab)
                    const double theta = (Gm[b][b] - Gm[a][a]) / (2.0 * apq);
                    const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
                    const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                    for (int k = 0; k < nz; ++k) {         // columns a, b
                        const double ga = Gm[k][a], gb = Gm[k][b];
                        Gm[k][a] = c * ga - sn * gb;
                        Gm[k][b] = sn * ga + c * gb;
                    }
                    for (int k = 0; k < nz; ++k) {         // rows a, b
                        const double ga = Gm[a][k], gb = Gm[b][k];
                        Gm[a][k] = c * ga - sn * gb;
                        Gm[b][k] = sn * ga + c * gb;
                    }
                    for (int k = 0; k < nz; ++k) {
                        const double va = Vm[k][a], vb = Vm[k][b];
                        Vm[k][a] = c * va - sn * vb;
                        Vm[k][b] = sn * va + c * vb;
                    }
                }
        }
        for (int a = 0; a < nz; ++a) {
            lam[a] = Gm[a][a];
            order[a] = a;
        }
        for (int a = 1; a < nz; ++a)             // descending eigenvalues
            for (int b = a; b > 0 && lam[order[b]] > lam[order[b - 1]]; --b) {
                const int tmp = order[b];
                order[b] = order[b - 1];
                order[b - 1] = tmp;
            }
        const double top = lam[order[0]];
        int kp = 0;
        while (kp < nz && top > 0.0 && lam[order[kp]] > eps1 * eps1 * top) ++kp;
        nkeep = kp;
    }
    __syncthreads();
    const int kp = nkeep;
    for (int i = tid; i < m; i += NT) {
        double zr[TRUNC_MAXZ];
#pragma unroll
        for (int a = 0; a < TRUNC_MAXZ; ++a) zr[a] = (a < nz) ? Z[i + size_t(a) * m] : 0.0;
        for (int c = 0; c < nz; ++c) {
            double v = 0.0;
            if (c < kp) {
                const int j = order[c];
#pragma unroll
                for (int a = 0; a < TRUNC_MAXZ; ++a)
                    if (a < nz) v += zr[a] * Vm[a][j];
                v /= sqrt(lam[j]);
            }
            Z[i + size_t(c) * m] = v;
        }
    }
}

void launch_gc_truncate(const CompressTask* d_tasks, int ntasks, double eps1, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_gc_truncate", 0.0, s);
    hipLaunchKernelGGL(k_gc_truncate, dim3(ntasks), dim3(NT), 0, s, d_tasks, eps1);
    check_launch("k_gc_truncate");
}

// Rayleigh-Ritz on a window W (m x s, s <= 16) of the basis: the last kept directions and the
// first ones past the threshold. One workgroup per node:
//   C = B B^T (s x s) from B = W^T A_sw (s x wt, ld s) on the FP64 matrix cores: the 16 x 16
//     product with K = 4 takes B's rows as both operands; the four waves take every fourth
//     group of four columns of B and their partial products are summed in LDS;
//   the eigenvectors of C by Jacobi in tournament order (eight disjoint rotations per step,
//     15 steps per sweep): rotation (p, q) zeroes c_pq (tan of the angle from
//     (c_qq - c_pp) / 2 c_pq, the smaller root); pairs with |c_pq| <= eps_mach sqrt(|c_pp c_qq|)
//     are skipped; sweeps end when none rotates (at most 30);
//   W's first w columns <- W times the eigenvectors of the w largest eigenvalues (each thread
//     reads and rewrites whole rows of W, so the product is in place).
__global__ __launch_bounds__(NT) void k_comp_ritz(const RitzTask* tasks) {
    typedef Mma<double> MM;
    constexpr int R = RITZ_MAX;
    static_assert(R == 16 && NT == 4 * WAVE, "one 16 x 16 matrix-core block per wave");
    __shared__ double cp[NT / WAVE][R][R + 1];
    __shared__ double a[R][R + 1], v[R][R + 1];
    __shared__ double rc[R / 2], rs[R / 2];
    __shared__ int rp[R / 2], rq[R / 2], inv[R], anyf[2];
    const RitzTask T = tasks[blockIdx.x];
    const int s = T.s, tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    {
        const HS_G double* B = gp(T.B);
        typename MM::acc acc = MM::zero();
        const int i = lane % 16;
        // eight groups of four columns per round, their loads issued before the products
        constexpr int UR = 8, STEP = 4 * (NT / WAVE);
        for (int k0 = 4 * wv; k0 < T.wt; k0 += UR * STEP) {
            double x[UR];
#pragma unroll
            for (int u = 0; u < UR; ++u) {
                const int kk = k0 + u * STEP + lane / 16;
                x[u] = (i < s && kk < T.wt) ? B[i + size_t(kk) * s] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UR; ++u) acc = MM::mac(x[u], x[u], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) cp[wv][MM::row(lane, r)][i] = acc[r];
    }
    __syncthreads();
    {
        const int i = tid % R, j = tid / R;                 // NT = R * R entries
        double c = 0.0;
#pragma unroll
        for (int w = 0; w < NT / WAVE; ++w) c += (i >= j) ? cp[w][i][j] : cp[w][j][i];
        a[i][j] = c;
        v[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // round r of the tournament: position 0 stays, the others rotate; pair i = (pos i, pos 15 - i)
    auto player = [](int pos, int r) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (R - 1); };
    // the "any rotation" flag of a sweep alternates between two slots: a slot is cleared again
    // only after every thread has passed the next sweep's first barrier, that is after its
    // read of the slot
    for (int sweep = 0; sweep < 30; ++sweep) {
        int* anyr = &anyf[sweep & 1];
        if (tid == 0) *anyr = 0;
        __syncthreads();
        for (int r = 0; r < R - 1; ++r) {
            if (tid < R / 2) {
                const int pa = player(tid, r), pb = player(R - 1 - tid, r);
                const int p = min(pa, pb), q = max(pa, pb);
                double c = 1.0, sn = 0.0;
                if (q < s) {
                    const double apq = a[p][q], app = a[p][p], aqq = a[q][q];
                    if (apq != 0.0 && fabs(apq) > DBL_EPSILON * sqrt(fabs(app * aqq))) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                        *anyr = 1;
                    }
                }
                rp[tid] = p;
                rq[tid] = q;
                rc[tid] = c;
                rs[tid] = sn;
            }
            __syncthreads();
            if (tid < R * R / 2) {                      // columns p, q of A and V, row j
                const int pi = tid / R, j = tid % R;
                const double c = rc[pi], sn = rs[pi];
                if (sn != 0.0) {
                    const int p = rp[pi], q = rq[pi];
                    const double ajp = a[j][p], ajq = a[j][q];
                    a[j][p] = c * ajp - sn * ajq;
                    a[j][q] = sn * ajp + c * ajq;
                    const double vjp = v[j][p], vjq = v[j][q];
                    v[j][p] = c * vjp - sn * vjq;
                    v[j][q] = sn * vjp + c * vjq;
                }
            }
            __syncthreads();
            if (tid < R * R / 2) {                      // rows p, q of A, column j
                const int pi = tid / R, j = tid % R;
                const double c = rc[pi], sn = rs[pi];
                if (sn != 0.0) {
                    const int p = rp[pi], q = rq[pi];
                    const double apj = a[p][j], aqj = a[q][j];
                    a[p][j] = c * apj - sn * aqj;
                    a[q][j] = sn * apj + c * aqj;
                }
            }
            __syncthreads();
        }
        if (*anyr == 0) break;                          // uniform: read after the barrier
    }
    if (tid < s) {
        const double li = a[tid][tid];
        int r = 0;
        for (int j = 0; j < s; ++j) {
            const double lj = a[j][j];
            r += (lj > li || (lj == li && j < tid)) ? 1 : 0;
        }
        inv[r] = tid;                                   // eigenvector of the r-th largest
    }
    __syncthreads();
    HS_G double* W = gp(T.W);
    for (int row = tid; row < T.m; row += NT) {
        double x[R];
#pragma unroll
        for (int c = 0; c < R; ++c) x[c] = (c < s) ? W[row + size_t(c) * T.ldw] : 0.0;
        for (int o = 0; o < T.w; ++o) {
            const int e = inv[o];
            double y = 0.0;
#pragma unroll
            for (int c = 0; c < R; ++c) y += x[c] * v[c][e];
            W[row + size_t(o) * T.ldw] = y;
        }
    }
}

void launch_comp_ritz(const RitzTask* d_tasks, int ntasks, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_comp_ritz", 0.0, s);
    hipLaunchKernelGGL(k_comp_ritz, dim3(ntasks), dim3(NT), 0, s, d_tasks);
    check_launch("k_comp_ritz");
}

void launch_compress(const CompressTask* d_tasks, int ntasks, int variant, double eps, int* d_rank,
                     int* d_extra, int kx_max, double flops, bool lds, int max_m, int force_lpe,
                     int force_vectors, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_m > CMP_MAX)
        throw Error{HSOLVE_ERR_INVALID, "super node larger than 512 unknowns at compression"};
    {
        ProfScope ps(lds ? "k_comp_reduce<true, 128>" : "k_comp_reduce<false, 512>", flops, s);
        if (lds) {
            if (max_m > CMP_LDS_MAX) throw Error{HSOLVE_ERR_INVALID, "internal: LDS compression too large"};
            static std::once_flag once;
            set_lds_limit(once, reinterpret_cast<const void*>(&k_comp_reduce<true, CMP_LDS_MAX>),
                          (size_t(CMP_LDS_MAX) * (CMP_LDS_MAX + 1) + 3 * CMP_LDS_MAX) * sizeof(double));
            // the matrix, then the register-resident tridiagonalisation's scratch
            const size_t bytes = (size_t(max_m) * (CMP_LDS_MAX + 1) + 3 * CMP_LDS_MAX) * sizeof(double);
            hipLaunchKernelGGL((k_comp_reduce<true, CMP_LDS_MAX>), dim3(ntasks), dim3(NT), bytes, s,
                               d_tasks, variant, eps, d_rank, d_extra, kx_max);
            check_launch("k_comp_reduce<lds>");
        } else {
            const size_t bytes = size_t(TRI_LDS_DOUBLES) * sizeof(double);
            static std::once_flag once;
            set_lds_limit(once, reinterpret_cast<const void*>(&k_comp_reduce<false, CMP_MAX>), bytes);
            hipLaunchKernelGGL((k_comp_reduce<false, CMP_MAX>), dim3(ntasks), dim3(CMP_GLOBAL_NT), bytes, s, d_tasks,
                               variant, eps, d_rank, d_extra, kx_max);
            check_launch("k_comp_reduce<global>");
        }
    }
    {
        ProfScope ps("k_comp_bisect", 0.0, s);
        // lanes per eigenvalue from the number of eigenvalues the launch can hold
        // lanes per eigenvalue: the widest group that keeps the launch within one wave per SIMD
        // (64 K lanes), so that a launch with few nodes still fills the chip
        const double total = double(max_m) * ntasks;
        int lpe = 64;
        while (lpe > 1 && total * lpe > 65536.0) lpe /= 2;
        if (force_lpe > 0) lpe = force_lpe;      // a fixed launch shape (tests, tuning)
        auto go = [&](auto kern, int l) {
            hipLaunchKernelGGL(kern, dim3((max_m + NT / l - 1) / (NT / l), ntasks), dim3(NT), 0, s, d_tasks);
        };
        switch (lpe) {
            case 64: go(k_comp_bisect<64>, 64); break;
            case 32: go(k_comp_bisect<32>, 32); break;
            case 16: go(k_comp_bisect<16>, 16); break;
            case 8: go(k_comp_bisect<8>, 8); break;
            case 4: go(k_comp_bisect<4>, 4); break;
            case 2: go(k_comp_bisect<2>, 2); break;
            default: go(k_comp_bisect<1>, 1); break;
        }
        check_launch("k_comp_bisect");
    }
    {
        ProfScope ps("k_comp_vectors", 0.0, s);
        const bool lane = force_vectors ? force_vectors == 1 : double(max_m) * ntasks >= 4096.0;
        if (lane) {                                  // many eigenvalues: one lane each
            hipLaunchKernelGGL(k_comp_vectors, dim3((max_m + VL - 1) / VL, ntasks), dim3(VL), 0, s, d_tasks);
        } else {                                     // few: one wave each (latency)
            const int ldn = max_m;
            const size_t bytes = sizeof(double) * (2 + 5 * (VNT / WAVE)) * size_t(ldn) +
                                 sizeof(int) * (VNT / WAVE) * size_t(ldn);
            hipLaunchKernelGGL(k_comp_vectors_wave, dim3((max_m + VNT / WAVE - 1) / (VNT / WAVE), ntasks),
                               dim3(VNT), bytes, s, d_tasks, ldn);
        }
        check_launch("k_comp_vectors");
    }
    {
        ProfScope ps("k_comp_orth", 0.0, s);
        hipLaunchKernelGGL(k_comp_orth, dim3((max_m + NT / WAVE - 1) / (NT / WAVE), ntasks), dim3(NT), 0, s,
                           d_tasks);
        check_launch("k_comp_orth");
    }
    {
        ProfScope ps("k_comp_wy", 0.0, s);
        hipLaunchKernelGGL(k_comp_wy, dim3((max_m + WY_NB - 1) / WY_NB, ntasks), dim3(NT), 0, s, d_tasks);
        check_launch("k_comp_wy");
    }
    {
        ProfScope ps("k_comp_bt", 0.0, s);
        const size_t bytes = sizeof(double) * (size_t(BT_COLS) * (max_m + 1) + size_t(WY_NB) * (max_m + 1) +
                                               WY_NB * BT_COLS + WY_NB * (WY_NB + 1) +
                                               (NT / WAVE) * WY_NB * BT_COLS);
        static std::once_flag once;
        set_lds_limit(once, reinterpret_cast<const void*>(&k_comp_bt),
                      sizeof(double) * (size_t(BT_COLS) * (CMP_MAX + 1) + size_t(WY_NB) * (CMP_MAX + 1) +
                                        WY_NB * BT_COLS + WY_NB * (WY_NB + 1) + (NT / WAVE) * WY_NB * BT_COLS));
        hipLaunchKernelGGL(k_comp_bt, dim3((max_m + BT_COLS - 1) / BT_COLS, ntasks), dim3(NT), bytes, s, d_tasks,
                           variant);
        check_launch("k_comp_bt");
    }
}

}  // namespace hs
