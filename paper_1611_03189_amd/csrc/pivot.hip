// Pivot blocks: Cholesky A = L L^T and the explicit inverse A^{-1} = L^{-T} L^{-1}, one
// workgroup per block. Used for A_ss^{-1} and S^{-1} (§3.2 elimination; Appendix A).
//
// k_chol_inv     blocks up to PIV_LDS_MAX rows, held in LDS with leading dimension m+1
//                (odd stride: the column walks of the inverse and of the product hit
//                distinct banks): right-looking Cholesky and in-place lower-triangular
//                inverse X = L^{-1} (column j = -(X22 l_j) / l_jj, right to left), two
//                barriers per column each, then A^{-1} = X^T X written to both triangles.
// k_chol_inv_blk larger blocks (up to PIV_MAX rows) in a global work matrix, blocked by
//                PIV_NB columns: the panel's diagonal block is factored and inverted in
//                one pass of steps in LDS, the panel below it (L21 = A21 L11^{-T}) and
//                the trailing update run on the matrix cores; the inverse is blocked the same
//                way (X21 = -X22 L21 X11, right to left, also on the matrix cores). X =
//                L^{-1} is left in the work matrix (upper triangle zeroed) for the product
//                A^{-1} = X^T X, which the caller forms with the grouped GEMM over many
//                workgroups.
#include "hs_device.h"

namespace hs {

constexpr int PIV_LDS_MAX = 128;
constexpr int PIV_MAX = 512;
constexpr int PIV_NB = 32;
constexpr int PIV_PANEL = PIV_MAX * PIV_NB;     // elements of the LDS panel buffer

template <typename R>
__global__ __launch_bounds__(NT) void k_chol_inv(const CholTask* tasks, int* fail) {
    extern __shared__ double lds_raw[];             // typed double: 8-byte aligned LDS accesses
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    R* W = reinterpret_cast<R*>(lds_raw);
    const int ldw = m + 1;
    const HS_G R* A = gp(static_cast<const R*>(T.A));
    HS_G R* Ainv = gp(static_cast<R*>(T.Ainv));
    copy_block(W, ldw, A, T.lda, m, m);
    __syncthreads();
    // two barriers per column: every thread takes the pivot sqrt(d_j) itself, the diagonal
    // entry is stored once the column is scaled (nobody reads it any more in this step)
    bool failed = false;
    for (int j = 0; j < m; ++j) {
        const R d = W[j + j * ldw];
        if (!(d > R(0)) || !isfinite(d)) {
            failed = true;                              // uniform: every thread read the same d
            break;
        }
        const R piv = sqrt(d);
        for (int i = j + 1 + tid; i < m; i += NT) W[i + j * ldw] /= piv;
        __syncthreads();
        if (tid == 0) W[j + j * ldw] = piv;
        // trailing update, rows over threads (the column-j entry of a row stays in a register)
        for (int i = j + 1 + tid; i < m; i += NT) {
            const R lij = W[i + j * ldw];
            int k = j + 1;
            for (; k + 4 <= i + 1; k += 4) {
                R t[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) t[u] = W[(k + u) + j * ldw];
#pragma unroll
                for (int u = 0; u < 4; ++u) W[i + (k + u) * ldw] -= lij * t[u];
            }
            for (; k <= i; ++k) W[i + k * ldw] -= lij * W[k + j * ldw];
        }
        __syncthreads();
    }
    if (failed) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }
    __syncthreads();
    // X = L^{-1} in place, columns right to left, two barriers per column: every thread takes
    // -1 / l_jj itself; X's column j and diagonal entry are stored once the column of L and
    // the old diagonal entry have been read
    for (int j = m - 1; j >= 0; --j) {
        const R ajj = -(R(1) / W[j + j * ldw]);
        R y = R(0);
        const int i = j + 1 + tid;         // m <= PIV_LDS_MAX < NT: at most one row per thread
        if (i < m) {
            R a[4] = {0, 0, 0, 0};
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
        if (tid == 0) W[j + j * ldw] = -ajj;
        __syncthreads();
    }
    // A^{-1} = X^T X
    for (int e = tid; e < m * m; e += NT) {
        const int i = e % m, j = e / m;
        if (i < j) continue;
        R s = R(0);
        for (int k = i; k < m; ++k) s += W[k + i * ldw] * W[k + j * ldw];
        Ainv[i + size_t(j) * T.ldi] = s;
        Ainv[j + size_t(i) * T.ldi] = s;
    }
}

// Cholesky of the nb x nb diagonal block at P (column-major, ld ldp, nb <= PIV_NB) in place
// and its inverse in X11 (full PIV_NB x PIV_NB, zeros above the diagonal and outside nb), by
// the whole workgroup: thread t owns the entries (t % 32, t / 32 + 8k), k < 4, of both. The
// factorisation keeps each column unscaled until the end (updates use a_rj a_cj / d_j); the
// forward substitution L X = I runs in the same steps, one barrier per step: at step j the
// column l_j = a_j / sqrt(d_j) is final, so the rows r > j of X take -l_rj X(j, :) / l_jj,
// and row r of X is divided by l_rr at the end. Sets *bad on a non-positive pivot (every
// thread sees the same pivot, so all leave together).
template <typename R>
__device__ void block_potrf_trinv32(R* P, int ldp, int nb, R* X11, int* bad) {
    constexpr int l11 = PIV_NB + 1;
    const int r = threadIdx.x % PIV_NB, cb = threadIdx.x / PIV_NB;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        X11[r + c * l11] = (r == c && r < nb) ? R(1) : R(0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const R dj = P[j + j * ldp];
        if (!(dj > R(0)) || !isfinite(dj)) {
            if (threadIdx.x == 0) *bad = 1;
            return;                                 // uniform: every thread read the same dj
        }
        const R idj = R(1) / dj;
        const R arj = (r < nb) ? P[r + j * ldp] : R(0);
        const R sdj = sqrt(dj), ilj = R(1) / sdj;
        const R lrj = (r > j && r < nb) ? arj / sdj : R(0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = cb + 8 * k;
            if (c > j && c <= r && r < nb) P[r + c * ldp] -= arj * P[c + j * ldp] * idj;
            if (r > j && r < nb && c <= j) X11[r + c * l11] -= lrj * X11[j + c * l11] * ilj;
        }
        __syncthreads();
    }
    // scale: L(r, c) = a_rc / sqrt(d_c), L(c, c) = sqrt(d_c); X's rows by 1 / L(r, r)
    const R sdr = (r < nb) ? sqrt(P[r + r * ldp]) : R(1);
    R l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        l[k] = R(0);
        if (r < nb && c < nb && c <= r) l[k] = (r == c) ? sdr : P[r + c * ldp] / sqrt(P[c + c * ldp]);
        if (r < nb) X11[r + c * l11] /= sdr;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = cb + 8 * k;
        if (r < nb && c < nb && c <= r) P[r + c * ldp] = l[k];
    }
    __syncthreads();
}

// rows [i_begin, i_end) of P (column-major, ld ldp, nb <= PIV_NB columns): P(i, :) <-
// P(i, :) X11^T (TRANS) or P(i, :) X11, X11 a full PIV_NB x PIV_NB matrix in LDS (zeros
// outside nb), on the matrix cores: each wave takes blocks of 16 rows (blocks w, w + 4, ..)
// as two 16 x 16 output blocks over K = 32 (lane l: operand A = P(i0 + l % 16, k), operand B
// = the X11 entry of (k, column 16 y + l % 16), k = 4 s + l / 16). A block's rows are read
// into the products before they are written back; rows past i_end are read clamped and not
// stored.
template <bool TRANS, typename R>
__device__ inline void rows_times_x11(R* P, int ldp, int i_begin, int i_end, int nb, const R* X11) {
    typedef Mma<R> MM;
    constexpr int l11 = PIV_NB + 1;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    const int li = lane % 16, lk = lane / 16;
    for (int i0 = i_begin + 16 * wv; i0 < i_end; i0 += 16 * (NT / WAVE)) {
        const int ia = min(i0 + li, i_end - 1);
        typename MM::acc acc[2] = {MM::zero(), MM::zero()};
#pragma unroll
        for (int s = 0; s < PIV_NB / 4; ++s) {
            const int k = 4 * s + lk;
            const R av = (k < nb) ? P[ia + k * ldp] : R(0);
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const int c = 16 * y + li;
                const R bv = TRANS ? X11[c + k * l11] : X11[k + c * l11];
                acc[y] = MM::mac(av, bv, acc[y]);
            }
        }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + MM::row(lane, u), c = 16 * y + li;
                if (i < i_end && c < nb) P[i + c * ldp] = acc[y][u];
            }
    }
}

template <typename R>
__global__ __launch_bounds__(NT) void k_chol_inv_blk(const CholTask* tasks, int* fail) {
    typedef Mma<R> MM;
    extern __shared__ double lds_raw[];             // typed double: 8-byte aligned LDS accesses
    R* Pn = reinterpret_cast<R*>(lds_raw);          // panel / Y buffer, PIV_PANEL elements
    __shared__ R X11[PIV_NB * (PIV_NB + 1)];
    __shared__ int bad;
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x;
    constexpr int l11 = PIV_NB + 1;
    HS_G R* W = gp(static_cast<R*>(T.work));       // m x m, ld m
    const HS_G R* A = gp(static_cast<const R*>(T.A));
    auto stamp = [&](int k) {
        if (T.tstamp && tid == 0) T.tstamp[k] = clock64();
    };
    stamp(0);
    const size_t ld = size_t(m);
    copy_block(W, ld, A, T.lda, m, m);
    if (tid == 0) bad = 0;
    __syncthreads();
    stamp(1);

    // trace only: cycles of the panel phases (copy, diagonal block, L21, write-back,
    // trailing update) summed over the panels into tstamp[4..8]
    long long pcyc[5] = {0, 0, 0, 0, 0}, tprev = 0;
    auto phase = [&](int k) {
        if (T.tstamp && tid == 0) {
            const long long tnow = clock64();
            if (k >= 0) pcyc[k] += tnow - tprev;
            tprev = tnow;
        }
    };
    // ---- blocked right-looking Cholesky; the diagonal blocks of W receive L11^{-1} ----
    for (int jb = 0; jb < m; jb += PIV_NB) {
        const int nb = min(PIV_NB, m - jb);
        const int r = m - jb;                        // panel rows (diagonal block first)
        phase(-1);
        copy_block(Pn, r, W + jb + jb * ld, ld, r, nb);
        __syncthreads();
        phase(0);
        // L11 and its inverse by the whole workgroup
        block_potrf_trinv32(Pn, r, nb, X11, &bad);
        __syncthreads();
        phase(1);
        if (bad) break;
        // L21 = A21 L11^{-T}, rows in registers
        rows_times_x11<true>(Pn, r, nb, r, nb, X11);
        __syncthreads();
        phase(2);
        for (int e = tid; e < r * nb; e += NT) {
            const int i = e % r, c = e / r;
            W[(jb + i) + (jb + c) * ld] = (i < nb) ? X11[i + c * l11] : Pn[i + c * r];
        }
        phase(3);
        // trailing update W22 -= L21 L21^T, L21 = Pn(nb.., :), on the FP64 matrix cores: the
        // 64 x 64 tiles on and below the diagonal (column of tiles by column), wave wv takes
        // the 32 x 32 quarter (rows 32 (wv % 2), columns 32 (wv / 2)) as 2 x 2 blocks of
        // v_mfma_f64_16x16x4f64 over K = nb. The product is formed transposed (operand A over
        // the tile's columns, B over its rows) so that lane l's accumulator register u is
        // W22(l % 16, l / 16 + 4 u) of its block. The next tile is loaded before the current
        // one is multiplied; rows and columns past the matrix are read clamped, never stored.
        {
            const int t = r - nb;
            const int Tb = (t + 63) / 64, ntile = Tb * (Tb + 1) / 2;
            const int lane = tid % WAVE, wv = tid / WAVE;
            const int li = lane % 16, lk = lane / 16;
            const int qr = 32 * (wv % 2), qc = 32 * (wv / 2);
            HS_G R* W22 = W + (jb + nb) + (jb + nb) * ld;
            int rr[2], cc[2][4], cbase[2];
            typename MM::acc nxt[2][2];
            auto tile_pos = [&](int bt) {
                int bj = 0, rem = bt;                 // column-major order of the lower tiles
                while (rem >= Tb - bj) {
                    rem -= Tb - bj;
                    ++bj;
                }
                const int bi = bj + rem;
#pragma unroll
                for (int x = 0; x < 2; ++x) rr[x] = 64 * bi + qr + 16 * x + li;
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cbase[y] = 64 * bj + qc + 16 * y;
#pragma unroll
                    for (int u = 0; u < 4; ++u) cc[y][u] = cbase[y] + MM::row(lane, u);
                }
            };
            auto load_tile = [&]() {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            nxt[x][y][u] = W22[min(rr[x], t - 1) + size_t(min(cc[y][u], t - 1)) * ld];
            };
            if (ntile > 0) {
                tile_pos(0);
                load_tile();
            }
            for (int bt = 0; bt < ntile; ++bt) {
                typename MM::acc acc[2][2];
                int r_cur[2], c_cur[2][4], cb_cur[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    r_cur[x] = rr[x];
#pragma unroll
                    for (int y = 0; y < 2; ++y) acc[x][y] = nxt[x][y];
                }
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    cb_cur[y] = cbase[y];
#pragma unroll
                    for (int u = 0; u < 4; ++u) c_cur[y][u] = cc[y][u];
                }
                int sa[2], rb[2];                       // panel rows of this lane's operands
#pragma unroll
                for (int y = 0; y < 2; ++y) sa[y] = nb + min(cb_cur[y] + li, t - 1);
#pragma unroll
                for (int x = 0; x < 2; ++x) rb[x] = nb + min(r_cur[x], t - 1);
                if (bt + 1 < ntile) {
                    tile_pos(bt + 1);
                    load_tile();
                }
                // all PIV_NB / 4 steps, unrolled (operands past nb are zero: the products
                // add exact zeros), so that the operand reads of a tile issue together
#pragma unroll
                for (int ks = 0; ks < PIV_NB / 4; ++ks) {
                    const int k = 4 * ks + lk;
                    const bool kv = k < nb;
                    const int kc = kv ? k : 0;
                    R a[2], b[2];
#pragma unroll
                    for (int y = 0; y < 2; ++y) a[y] = kv ? -Pn[sa[y] + kc * r] : R(0);
#pragma unroll
                    for (int x = 0; x < 2; ++x) b[x] = kv ? Pn[rb[x] + kc * r] : R(0);
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 2; ++y) acc[x][y] = MM::mac(a[y], b[x], acc[x][y]);
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (r_cur[x] < t && c_cur[y][u] < t) W22[r_cur[x] + size_t(c_cur[y][u]) * ld] = acc[x][y][u];
            }
        }
        __syncthreads();
        phase(4);
    }
    if (T.tstamp && tid == 0)
        for (int k = 0; k < 5; ++k) T.tstamp[4 + k] = pcyc[k];
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
            X11[i + c * l11] = (i < nb && c < nb && i >= c) ? W[(jb + i) + (jb + c) * ld] : R(0);
        }
        copy_block(Pn, t, W + (jb + nb) + jb * ld, ld, t, nb);
        __syncthreads();
        rows_times_x11<false>(Pn, t, 0, t, nb, X11);     // Y = L21 X11
        __syncthreads();
        // X21 = -X22 Y on the FP64 matrix cores, X22 = the lower-triangular inverse already in W
        // (its stale upper part is masked): 64-row blocks of X21, wave wv takes rows 16 wv ..
        // 16 wv + 15 of the block and the nb <= 32 columns as two 16 x 16 blocks; K runs over
        // the columns l of X22 up to the block's last row. Formed transposed (operand A over
        // the columns of Y, B over the rows of X22) so that lane l's register u is
        // X21(l % 16, l / 16 + 4 u) of its block. Four K steps are loaded ahead.
        {
            const int lane = tid % WAVE, wv = tid / WAVE;
            const int li = lane % 16, lk = lane / 16;
            const HS_G R* X22 = W + (jb + nb) + (jb + nb) * ld;
            for (int i0 = 0; i0 < t; i0 += 64) {
                const int i = i0 + 16 * wv + li;             // this lane's row (operand B)
                const int ic = min(i, t - 1);
                const int kend = min(i0 + 64, t);
                const int nks = (kend + 3) / 4;
                typename MM::acc acc[2] = {MM::zero(), MM::zero()};
                auto ldb = [&](int ks) {
                    const int l = 4 * ks + lk;
                    return (l < kend && l <= i && i < t) ? X22[ic + size_t(min(l, t - 1)) * ld] : R(0);
                };
                R bq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) bq[q] = ldb(q);
                for (int ks0 = 0; ks0 < nks; ks0 += 4) {
                    R bc[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) bc[q] = bq[q];
#pragma unroll
                    for (int q = 0; q < 4; ++q) bq[q] = ldb(ks0 + 4 + q);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int l = 4 * (ks0 + q) + lk;
                        const int lc = min(l, t - 1);
#pragma unroll
                        for (int y = 0; y < 2; ++y) {
                            const int c = 16 * y + li;
                            const R av = (l < kend && c < nb) ? Pn[lc + min(c, nb - 1) * t] : R(0);
                            acc[y] = MM::mac(av, bc[q], acc[y]);
                        }
                    }
                }
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int c = 16 * y + MM::row(lane, u);
                        if (i < t && c < nb) W[(jb + nb + i) + (jb + c) * ld] = -acc[y][u];
                    }
            }
        }
        __syncthreads();
    }
    // upper triangle of X is zero for the product X^T X
    for (size_t e = tid; e < ld * m; e += NT) {
        const size_t i = e % ld, j = e / ld;
        if (i < j) W[e] = R(0);
    }
    stamp(3);
}

template <typename R>
void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops, bool lds,
                     int max_m, hipStream_t s) {
    if (ntasks <= 0) return;
    if (max_m > PIV_MAX) throw Error{HSOLVE_ERR_INVALID, "pivot block larger than 512"};
    const bool f32 = sizeof(R) == 4;
    ProfScope ps(lds ? (f32 ? "k_chol_inv_f32" : "k_chol_inv") : (f32 ? "k_chol_inv_blk_f32" : "k_chol_inv_blk"),
                 flops, s);
    if (lds) {
        if (max_m > PIV_LDS_MAX) throw Error{HSOLVE_ERR_INVALID, "internal: LDS pivot too large"};
        const size_t bytes = size_t(max_m) * (max_m + 1) * sizeof(R);
        static std::once_flag once;
        set_lds_limit(once, reinterpret_cast<const void*>(&k_chol_inv<R>),
                      size_t(PIV_LDS_MAX) * (PIV_LDS_MAX + 1) * sizeof(R));
        hipLaunchKernelGGL(k_chol_inv<R>, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv");
    } else {
        const size_t bytes = size_t(PIV_PANEL) * sizeof(R);
        static std::once_flag once;
        set_lds_limit(once, reinterpret_cast<const void*>(&k_chol_inv_blk<R>), bytes);
        hipLaunchKernelGGL(k_chol_inv_blk<R>, dim3(ntasks), dim3(NT), bytes, s, d_tasks, d_fail);
        check_launch("k_chol_inv_blk");
    }
}
template void launch_chol_inv<double>(const CholTask*, int, int*, double, bool, int, hipStream_t);
template void launch_chol_inv<float>(const CholTask*, int, int*, double, bool, int, hipStream_t);

}  // namespace hs
