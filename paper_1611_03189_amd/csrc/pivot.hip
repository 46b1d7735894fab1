// Pivot blocks: Cholesky A = L L^T and the explicit inverse A^{-1} = L^{-T} L^{-1}, one
// workgroup per block. Used for A_ss^{-1} and S^{-1} (§3.2 elimination; Appendix A).
//
// k_chol_inv     blocks up to PIV_LDS_MAX rows, held in LDS with leading dimension m+1
//                (odd stride: the column walks of the inverse and of the product hit
//                distinct banks): right-looking Cholesky, in-place lower-triangular
//                inverse X = L^{-1} (column j = -(X22 l_j) / l_jj, right to left), then
//                A^{-1} = X^T X written to both triangles.
// k_chol_inv_blk larger blocks (up to PIV_MAX rows) in a global work matrix, blocked by
//                PIV_NB columns: the current panel is factored in LDS, the trailing
//                matrix is updated with 4x4 register tiles; the inverse is blocked the
//                same way (X21 = -X22 L21 X11, right to left). X = L^{-1} is left in the
//                work matrix (upper triangle zeroed) for the product A^{-1} = X^T X, which
//                the caller forms with the grouped GEMM over many workgroups.
#include "hs_device.h"

namespace hs {

constexpr int PIV_LDS_MAX = 128;
constexpr int PIV_MAX = 512;
constexpr int PIV_NB = 32;
constexpr int PIV_PANEL = PIV_MAX * PIV_NB;     // doubles of the LDS panel buffer

__global__ __launch_bounds__(NT) void k_chol_inv(const CholTask* tasks, int* fail) {
    extern __shared__ double lds[];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    double* W = lds;
    const int ldw = m + 1;
    const HS_G double* A = gp(T.A);
    HS_G double* Ainv = gp(T.Ainv);
    copy_block(W, ldw, A, T.lda, m, m);
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double d = W[j + j * ldw];
            if (!(d > 0.0) || !isfinite(d)) bad = 1;
            else W[j + j * ldw] = sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        const double piv = W[j + j * ldw];
        for (int i = j + 1 + tid; i < m; i += NT) W[i + j * ldw] /= piv;
        __syncthreads();
        // trailing update, rows over threads (the column-j entry of a row stays in a register)
        for (int i = j + 1 + tid; i < m; i += NT) {
            const double lij = W[i + j * ldw];
            int k = j + 1;
            for (; k + 4 <= i + 1; k += 4) {
                double t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = W[(k + u) + j * ldw];
#pragma unroll
                for (int u = 0; u < 4; ++u) W[i + (k + u) * ldw] -= lij * t[u];
            }
            for (; k <= i; ++k) W[i + k * ldw] -= lij * W[k + j * ldw];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }
    // X = L^{-1} in place, columns right to left
    for (int j = m - 1; j >= 0; --j) {
        if (tid == 0) W[j + j * ldw] = 1.0 / W[j + j * ldw];
        __syncthreads();
        const double ajj = -W[j + j * ldw];
        double y = 0.0;
        const int i = j + 1 + tid;         // m <= PIV_LDS_MAX < NT: at most one row per thread
        if (i < m) {
            double a[4] = {0, 0, 0, 0};
            int l = j + 1;
            for (; l + 4 <= i + 1; l += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] += W[i + (l + u) * ldw] * W[(l + u) + j * ldw];
            }
            for (; l <= i; ++l) a[0] += W[i + l * ldw] * W[l + j * ldw];
            y = (a[0] + a[1]) + (a[2] + a[3]);
        }
        __syncthreads();
        if (i < m) W[i + j * ldw] = ajj * y;
        __syncthreads();
    }
    // A^{-1} = X^T X
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i < j) continue;
        double s = 0.0;
        for (int k = i; k < m; ++k) s += W[k + i * ldw] * W[k + j * ldw];
        Ainv[i + size_t(j) * T.ldi] = s;
        Ainv[j + size_t(i) * T.ldi] = s;
    }
}


// Cholesky of the nb x nb diagonal block at P (column-major, ld ldp, nb <= PIV_NB) in place
// and its inverse in X11 (full PIV_NB x PIV_NB, zeros above the diagonal and outside nb), by
// the whole workgroup: thread t owns the entries (t % 32, t / 32 + 8k), k < 4. The
// factorisation keeps each column unscaled until the end (updates use a_rj a_cj / d_j),
// and the inverse solves L X = I by columns, one barrier per step. Sets *bad on a
// non-positive pivot (every thread sees the same pivot, so all leave together).
__device__ void block_potrf_trinv32(double* P, int ldp, int nb, double* X11, int* bad) {
    constexpr int l11 = PIV_NB + 1;
    const int r = threadIdx.x % PIV_NB, cb = threadIdx.x / PIV_NB;
    for (int j = 0; j < nb; ++j) {
        const double dj = P[j + j * ldp];
        if (!(dj > 0.0) || !isfinite(dj)) {
            if (threadIdx.x == 0) *bad = 1;
            return;                                 // uniform: every thread read the same dj
        }
        const double idj = 1.0 / dj;
        const double arj = (r < nb) ? P[r + j * ldp] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = cb + 8 * k;
            if (c > j && c <= r && r < nb) P[r + c * ldp] -= arj * P[c + j * ldp] * idj;
        }
        __syncthreads();
    }
    // scale: L(r, c) = a_rc / sqrt(d_c), L(c, c) = sqrt(d_c); X11 = I
    double l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        l[k] = 0.0;
        if (r < nb && c < nb && c <= r) l[k] = (r == c) ? sqrt(P[c + c * ldp]) : P[r + c * ldp] / sqrt(P[c + c * ldp]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        if (r < nb && c < nb && c <= r) P[r + c * ldp] = l[k];
        X11[r + c * l11] = (r == c && r < nb) ? 1.0 : 0.0;
    }
    __syncthreads();
    // forward substitution L X = I, columns in parallel; row j of X is scaled at the end
    for (int j = 0; j < nb; ++j) {
        const double ilj = 1.0 / P[j + j * ldp];
        const double lrj = (r > j && r < nb) ? P[r + j * ldp] : 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = cb + 8 * k;
            if (r > j && r < nb && c <= j) X11[r + c * l11] -= lrj * X11[j + c * l11] * ilj;
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        if (r < nb) X11[r + c * l11] /= P[r + r * ldp];
    }
    __syncthreads();
}

// rows [i_begin, i_end) of P (column-major, ld ldp): P(i, :) <- P(i, :) X11^T (trans) or
// P(i, :) X11, X11 a full PIV_NB x PIV_NB matrix in LDS; the row is held in registers
template <bool TRANS>
__device__ inline void rows_times_x11(double* P, int ldp, int i_begin, int i_end, int nb, const double* X11) {
    constexpr int l11 = PIV_NB + 1;
    for (int i = i_begin + threadIdx.x; i < i_end; i += NT) {
        double a[PIV_NB];
#pragma unroll
        for (int l = 0; l < PIV_NB; ++l) a[l] = (l < nb) ? P[i + l * ldp] : 0.0;
#pragma unroll 1
        for (int c = 0; c < nb; ++c) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < PIV_NB; ++l) s += a[l] * (TRANS ? X11[c + l * l11] : X11[l + c * l11]);
            P[i + c * ldp] = s;
        }
    }
}

__global__ __launch_bounds__(NT) void k_chol_inv_blk(const CholTask* tasks, int* fail) {
    extern __shared__ double Pn[];                  // panel / Y buffer, PIV_PANEL doubles
    __shared__ double X11[PIV_NB * (PIV_NB + 1)];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    constexpr int l11 = PIV_NB + 1;
    HS_G double* W = gp(T.work);                   // m x m, ld m
    const HS_G double* A = gp(T.A);
    auto stamp = [&](int k) {
        if (T.tstamp && tid == 0) T.tstamp[k] = clock64();
    };
    stamp(0);
    const size_t ld = size_t(m);
    copy_block(W, ld, A, T.lda, m, m);
    if (tid == 0) bad = 0;
    __syncthreads();
    stamp(1);

    // ---- blocked right-looking Cholesky; the diagonal blocks of W receive L11^{-1} ----
    for (int jb = 0; jb < m; jb += PIV_NB) {
        const int nb = min(PIV_NB, m - jb);
        const int r = m - jb;                        // panel rows (diagonal block first)
        copy_block(Pn, r, W + jb + jb * ld, ld, r, nb);
        __syncthreads();
        // L11 and its inverse by the whole workgroup
        block_potrf_trinv32(Pn, r, nb, X11, &bad);
        __syncthreads();
        if (bad) break;
        // L21 = A21 L11^{-T}, rows in registers
        rows_times_x11<true>(Pn, r, nb, r, nb, X11);
        __syncthreads();
        for (int e = tid; e < r * nb; e += NT) {
            const int i = e % r, c = e / r;
            W[(jb + i) + (jb + c) * ld] = (i < nb) ? X11[i + c * l11] : Pn[i + c * r];
        }
        // trailing update W22 -= L21 L21^T, L21 = Pn(nb.., :): 64 x 64 block tiles on and below
        // the diagonal, thread (tx, ty) of 16 x 16 takes rows tx + 16u and columns ty + 16w;
        // the next tile is loaded before the current one is computed
        {
            const int t = r - nb;
            const int Tb = (t + 63) / 64, ntile = Tb * (Tb + 1) / 2;
            const int tx = tid % 16, ty = tid / 16;
            auto tile_rc = [&](int bt, int* pr, int* pc, bool* okr, bool* okc) {
                int bj = 0, rem = bt;                 // column-major order of the lower tiles
                while (rem >= Tb - bj) {
                    rem -= Tb - bj;
                    ++bj;
                }
                const int bi = bj + rem;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ii = 64 * bi + tx + 16 * u, jj = 64 * bj + ty + 16 * u;
                    okr[u] = ii < t;
                    okc[u] = jj < t;
                    pr[u] = nb + min(ii, t - 1);      // panel rows (clamped)
                    pc[u] = nb + min(jj, t - 1);
                }
            };
            int pr[4], pc[4], prn[4], pcn[4];
            bool okr[4], okc[4], okrn[4], okcn[4];
            double nxt[4][4];
            if (ntile > 0) {
                tile_rc(0, prn, pcn, okrn, okcn);
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) nxt[u][v] = W[(jb + prn[u]) + (jb + pcn[v]) * ld];
            }
            for (int bt = 0; bt < ntile; ++bt) {
                double acc[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    pr[u] = prn[u];
                    pc[u] = pcn[u];
                    okr[u] = okrn[u];
                    okc[u] = okcn[u];
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = nxt[u][v];
                }
                if (bt + 1 < ntile) {
                    tile_rc(bt + 1, prn, pcn, okrn, okcn);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) nxt[u][v] = W[(jb + prn[u]) + (jb + pcn[v]) * ld];
                }
#pragma unroll 2
                for (int k = 0; k < nb; ++k) {
                    double a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u] = Pn[pr[u] + k * r];
                        b[u] = Pn[pc[u] + k * r];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] -= a[u] * b[v];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (okr[u] && okc[v]) W[(jb + pr[u]) + (jb + pc[v]) * ld] = acc[u][v];
            }
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }

    stamp(2);
    // ---- blocked inverse X = L^{-1}, panels right to left: X21 = -X22 L21 X11 ----
    const int last = ((m - 1) / PIV_NB) * PIV_NB;
    for (int jb = last; jb >= 0; jb -= PIV_NB) {
        const int nb = min(PIV_NB, m - jb);
        const int t = m - jb - nb;
        if (t == 0) continue;                      // the last diagonal block holds X11 already
        for (int e = tid; e < PIV_NB * PIV_NB; e += NT) {
            const int i = e % PIV_NB, c = e / PIV_NB;
            X11[i + c * l11] = (i < nb && c < nb && i >= c) ? W[(jb + i) + (jb + c) * ld] : 0.0;
        }
        copy_block(Pn, t, W + (jb + nb) + jb * ld, ld, t, nb);
        __syncthreads();
        rows_times_x11<false>(Pn, t, 0, t, nb, X11);     // Y = L21 X11
        __syncthreads();
        // X21 = -X22 Y, X22 = the lower-triangular inverse already in W; tiles of 4 rows x 8 cols
        const int Tr = (t + 3) / 4, Tc = (nb + 7) / 8;
        for (int idx = tid; idx < Tr * Tc; idx += NT) {
            const int i0 = 4 * (idx % Tr), c0 = 8 * (idx / Tr);
            double acc[4][8];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[u][v] = 0.0;
            const HS_G double* X22 = W + (jb + nb) + (jb + nb) * ld;
            // columns l <= i0: every row of the tile takes part. Rows past t and columns
            // past nb read clamped (in-bounds) entries; their sums are never stored.
            int xr[4], yc[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) xr[u] = min(i0 + u, t - 1);
#pragma unroll
            for (int v = 0; v < 8; ++v) yc[v] = min(c0 + v, nb - 1) * t;
            const int lend = min(i0, t - 1);
            int l = 0;
            if (l + 3 <= lend) {
                double xn[4][4];                    // next batch of columns, loaded ahead
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u) xn[q][u] = X22[xr[u] + size_t(l + q) * ld];
                for (; l + 3 <= lend; l += 4) {
                    double x[4][4], y[4][8];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int u = 0; u < 4; ++u) x[q][u] = xn[q][u];
                    if (l + 7 <= lend) {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int u = 0; u < 4; ++u) xn[q][u] = X22[xr[u] + size_t(l + 4 + q) * ld];
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int v = 0; v < 8; ++v) y[q][v] = Pn[l + q + yc[v]];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int v = 0; v < 8; ++v) acc[u][v] += x[q][u] * y[q][v];
                }
            }
            for (; l <= lend; ++l) {
                double x[4], y[8];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = X22[xr[u] + size_t(l) * ld];
#pragma unroll
                for (int v = 0; v < 8; ++v) y[v] = Pn[l + yc[v]];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 8; ++v) acc[u][v] += x[u] * y[v];
            }
            // columns i0 < l <= i0 + 3: only rows u with l <= i0 + u
            for (int l2 = i0 + 1; l2 <= i0 + 3 && l2 < t; ++l2) {
                double x[4], y[8];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    x[u] = (i0 + u < t && l2 <= i0 + u) ? X22[(i0 + u) + size_t(l2) * ld] : 0.0;
#pragma unroll
                for (int v = 0; v < 8; ++v) y[v] = (c0 + v < nb) ? Pn[l2 + (c0 + v) * t] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 8; ++v) acc[u][v] += x[u] * y[v];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    if (i0 + u < t && c0 + v < nb) W[(jb + nb + i0 + u) + (jb + c0 + v) * ld] = -acc[u][v];
        }
        __syncthreads();
    }
    // upper triangle of X is zero for the product X^T X
    for (size_t e = tid; e < ld * m; e += NT) {
        const size_t i = e % ld, j = e / ld;
        if (i < j) W[e] = 0.0;
    }
    stamp(3);
}

void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops, bool lds,
                     int max_m, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_m > PIV_MAX) throw Error{HSOLVE_ERR_INVALID, "pivot block larger than 512"};
    ProfScope ps(lds ? "k_chol_inv" : "k_chol_inv_blk", flops, s);
    if (lds) {
        if (max_m > PIV_LDS_MAX) throw Error{HSOLVE_ERR_INVALID, "internal: LDS pivot too large"};
        const size_t bytes = size_t(max_m) * (max_m + 1) * sizeof(double);
        static std::once_flag once;
        set_lds_limit(once, reinterpret_cast<const void*>(&k_chol_inv),
                      size_t(PIV_LDS_MAX) * (PIV_LDS_MAX + 1) * sizeof(double));
        hipLaunchKernelGGL(k_chol_inv, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv");
    } else {
        const size_t bytes = size_t(PIV_PANEL) * sizeof(double);
        static std::once_flag once;
        set_lds_limit(once, reinterpret_cast<const void*>(&k_chol_inv_blk), bytes);
        hipLaunchKernelGGL(k_chol_inv_blk, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv_blk");
    }
}

}  // namespace hs
