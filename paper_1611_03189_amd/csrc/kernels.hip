// HIP kernels for gfx950 (wave64). FP64 throughout.
//
//  k_copy        batched 2-D block copies (optional transpose)          block gather / merge
//  k_gemm        grouped GEMM over tile lists, C = bC + a sum op(A)op(B) Gram, Schur, T_N, L_nr, R
//  (pivot.hip: k_chol_inv*; compress.hip: k_comp_*)
//  k_fwd / k_bwd level sweeps of the solve phase                        apply
//  k_spmv, gathers/scatters (batched PCG kernels: krylov.hip)             outer PCG
#include <cfloat>

#include <algorithm>
#include <atomic>

#include "hs_device.h"

namespace hs {

// ---------------------------------------------------------------------------------
// Copies
// ---------------------------------------------------------------------------------
// One workgroup per COPY_COLS columns of the destination of one task (blockIdx.y), so that
// large blocks spread over many CUs.
constexpr int COPY_COLS = 32;

template <typename T>
__global__ __launch_bounds__(NT) void k_copy(const CopyTask* tasks) {
    const CopyTask t = tasks[blockIdx.x];
    const int j0 = blockIdx.y * COPY_COLS;
    if (j0 >= t.cols) return;
    const int nc = min(COPY_COLS, t.cols - j0);
    const HS_G T* src = gp(static_cast<const T*>(t.src));
    HS_G T* dst = gp(static_cast<T*>(t.dst));
    __shared__ T tile[32][33];
    if (!t.trans) {
        copy_block(dst + size_t(j0) * t.ldd, t.ldd, src + size_t(j0) * t.lds, t.lds, t.rows, nc);
        return;
    }
    // dst(i, j) = src(j, i) for the columns j0 .. j0 + nc of dst, through 32 x 32 tiles
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    for (int i0 = 0; i0 < t.rows; i0 += 32) {
        for (int r = ty; r < 32; r += 8) {
            const int si = j0 + tx, sj = i0 + r;               // src(si, sj), si < cols, sj < rows
            if (tx < nc && sj < t.rows) tile[r][tx] = src[si + size_t(sj) * t.lds];
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int di = i0 + tx, dj = j0 + r;               // dst(di, dj) = src(dj, di)
            if (di < t.rows && r < nc) dst[di + size_t(dj) * t.ldd] = tile[tx][r];
        }
        __syncthreads();
    }
}

template <typename T>
void launch_copy(const CopyTask* d_tasks, int ntasks, int max_cols, double bytes, hipStream_t s) {
    if (ntasks <= 0 || max_cols <= 0) return;
    ProfScope ps(sizeof(T) == 8 ? "k_copy" : "k_copy_f32", bytes, s);
    hipLaunchKernelGGL(k_copy<T>, dim3(ntasks, (max_cols + COPY_COLS - 1) / COPY_COLS), dim3(NT), 0, s, d_tasks);
    check_launch("k_copy");
}
template void launch_copy<double>(const CopyTask*, int, int, double, hipStream_t);
template void launch_copy<float>(const CopyTask*, int, int, double, hipStream_t);

// dst[i] = double(src[i]) for each task (the FP32 factorization's Gram matrices and kept
// vectors, read by the FP64 eigen-solver)
__global__ void k_promote(const PromoteTask* tasks) {
    const PromoteTask t = tasks[blockIdx.y];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < t.count;
         i += (long long)gridDim.x * blockDim.x)
        t.dst[i] = double(t.src[i]);
}

void launch_promote(const PromoteTask* d_tasks, int ntasks, double elems, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_promote", 12.0 * elems, s);
    hipLaunchKernelGGL(k_promote, dim3(64, ntasks), dim3(NT), 0, s, d_tasks);
    check_launch("k_promote");
}

// ---------------------------------------------------------------------------------
// Grouped GEMM on the FP64 matrix cores: TM x TN output tiles, 256 threads (4 waves in a
// 2 x 2 grid, each (TM/2) x (TN/2) = BX x BY blocks of v_mfma_f64_16x16x4f64), K in steps of
// TK through two LDS buffers, the next K step loaded into registers while the current one is
// multiplied. Every shape adds the k products of an output element in the same order (k
// ascending, four per instruction), so all shapes give the same bits; the autotuner picks
// one per size bucket.
// Operand layout of the instruction (per lane l of the wave): A(l % 16, l / 16),
// B(l / 16, l % 16); result register r holds C(l / 16 + 4 r, l % 16).
// ---------------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

struct GemmStep {            // position in the concatenated K loop of a task's terms
    int term, k0;
};

// REL: the flagged form of the apply sweeps (relative B and C addresses, negated terms, a
// column count per launch); without it the flags are ignored and none of that is compiled in.
template <typename T, int TM, int TN, int TK, bool REL>
__device__ inline void gemm_tile(const GemmTask* tasks, const GemmTerm* terms, const GemmTile tl,
                                 T (&As)[2][TK][TM + 1], T (&Bs)[2][TK][TN + 1], T* base0, T* base1,
                                 int ncols) {
    typedef Mma<T> MM;
    constexpr int BX = TM / 32, BY = TN / 32;              // 16 x 16 blocks per wave
    constexpr int LA = TM * TK / NT, LB = TN * TK / NT;    // loads per thread and K step
    static_assert(LA * NT == TM * TK && LB * NT == TN * TK, "tile");
    const GemmTask Tk = tasks[tl.task];
    const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    const int i0 = tl.ti * TM, j0 = tl.tj * TN;
    const int Nc = (REL && ncols > 0) ? ncols : Tk.N;      // columns of this launch
    if (REL && j0 >= Nc) return;
    typename MM::acc acc[BX][BY];
#pragma unroll
    for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < BY; ++y) acc[x][y] = MM::zero();

    T ra[LA], rb[LB];
    auto load_step = [&](GemmStep st) {
        const GemmTerm g = terms[st.term];
        const HS_G T* gA = gp(static_cast<const T*>(g.A));
        const HS_G T* gB = gp((REL && (g.flags & GEMM_REL))
                                  ? ((g.flags & GEMM_BASE1) ? base1 : base0) + reinterpret_cast<uintptr_t>(g.B)
                                  : static_cast<const T*>(g.B));
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + NT * q;
            int ii, kk;
            if (!g.transA) { ii = e % TM; kk = e / TM; } else { kk = e % TK; ii = e / TK; }
            const int gi = i0 + ii, gk = st.k0 + kk;
            ra[q] = (gi < Tk.M && gk < g.K) ? (g.transA ? gA[gk + size_t(gi) * g.lda] : gA[gi + size_t(gk) * g.lda])
                                            : T(0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + NT * q;
            int jj, kb;
            if (g.transB) { jj = e % TN; kb = e / TN; } else { kb = e % TK; jj = e / TK; }
            const int gj = j0 + jj, gkb = st.k0 + kb;
            rb[q] = (gj < Nc && gkb < g.K) ? (g.transB ? gB[gj + size_t(gkb) * g.ldb] : gB[gkb + size_t(gj) * g.ldb])
                                           : T(0);
        }
    };
    auto store_step = [&](GemmStep st, int buf) {
        const GemmTerm g = terms[st.term];
        // a negative term's sign goes on at the store, when the prefetched values are in
        // (on the load it would make the prefetch wait)
        const bool neg = REL && (g.flags & GEMM_NEG) != 0;
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int e = tid + NT * q;
            int ii, kk;
            if (!g.transA) { ii = e % TM; kk = e / TM; } else { kk = e % TK; ii = e / TK; }
            As[buf][kk][ii] = neg ? -ra[q] : ra[q];
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            const int e = tid + NT * q;
            int jj, kb;
            if (g.transB) { jj = e % TN; kb = e / TN; } else { kb = e % TK; jj = e / TK; }
            Bs[buf][kb][jj] = rb[q];
        }
    };
    auto next_step = [&](GemmStep st) {
        st.k0 += TK;
        while (st.term < Tk.t_end && st.k0 >= terms[st.term].K) {
            ++st.term;
            st.k0 = 0;
        }
        return st;
    };
    GemmStep cur{Tk.t_begin, 0};
    while (cur.term < Tk.t_end && terms[cur.term].K <= 0) ++cur.term;
    const int wr = (wv / 2) * (TM / 2), wc = (wv % 2) * (TN / 2);    // this wave's sub-tile
    const int fr = lane % 16, fk = lane / 16;
    int buf = 0;
    if (cur.term < Tk.t_end) load_step(cur);
    while (cur.term < Tk.t_end) {
        store_step(cur, buf);
        __syncthreads();
        const GemmStep nxt = next_step(cur);
        if (nxt.term < Tk.t_end) load_step(nxt);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 4) {
            T af[BX], bf[BY];
#pragma unroll
            for (int x = 0; x < BX; ++x) af[x] = As[buf][kk + fk][wr + 16 * x + fr];
#pragma unroll
            for (int y = 0; y < BY; ++y) bf[y] = Bs[buf][kk + fk][wc + 16 * y + fr];
#pragma unroll
            for (int x = 0; x < BX; ++x)
#pragma unroll
                for (int y = 0; y < BY; ++y)
                    acc[x][y] = MM::mac(af[x], bf[y], acc[x][y]);
        }
        cur = nxt;
        buf ^= 1;
    }
    HS_G T* C = gp((REL && (Tk.flags & GEMM_REL)) ? ((Tk.flags & GEMM_BASE1) ? base1 : base0) + reinterpret_cast<uintptr_t>(Tk.C)
                                          : static_cast<T*>(Tk.C));
    const T alpha = T(Tk.alpha), beta = T(Tk.beta);
#pragma unroll
    for (int x = 0; x < BX; ++x)
#pragma unroll
        for (int y = 0; y < BY; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wr + 16 * x + MM::row(lane, r), j = j0 + wc + 16 * y + fr;
                if (i < Tk.M && j < Nc) {
                    HS_G T* c = C + i + size_t(j) * Tk.ldc;
                    const T old = (Tk.beta == 0.0) ? T(0) : beta * (*c);
                    const T val = old + alpha * acc[x][y][r];
                    *c = val;
                    // (j, i) lies in a tile that is not listed: write its value there too
                    if ((Tk.flags & GEMM_MIRROR) && (i / TN) * TN >= (j / TM) * TM + TM)
                        C[j + size_t(i) * Tk.ldc] = val;
                }
            }
}

// One workgroup per tile, or, in the persistent form, a grid of resident workgroups that take
// tiles w, w + grid, .. of the list (the same computation per tile).
template <typename T, int TM, int TN, int TK, bool REL>
__global__ __launch_bounds__(NT) void k_gemm(const GemmTask* tasks, const GemmTerm* terms,
                                             const GemmTile* tiles, int ntiles, T* base0, T* base1, int ncols) {
    __shared__ T As[2][TK][TM + 1];
    __shared__ T Bs[2][TK][TN + 1];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        gemm_tile<T, TM, TN, TK, REL>(tasks, terms, tiles[t], As, Bs, base0, base1, ncols);
        __syncthreads();                           // the next tile refills the LDS buffers
    }
}

// 32 x 32 tiles with long K steps: four times the workgroups of a 64 x 64 tiling for launches
// with fewer tiles than compute units, each with a quarter of the tile's matrix-core work.
// The last two shapes run persistent: as many workgroups as fit on the chip at once, each
// looping over the tile list.
const GemmShape GEMM_SHAPES[GEMM_VARIANTS] = {{64, 64, 16, 0},   {64, 64, 32, 0}, {128, 64, 16, 0},
                                              {128, 128, 16, 0}, {32, 32, 64, 0}, {32, 32, 128, 0},
                                              {64, 64, 16, 1},   {32, 32, 64, 1}};

// resident workgroups of a kernel on this device (the persistent grid), found once per kernel
template <typename T, int TM, int TN, int TK>
static int resident_grid() {
    static std::atomic<int> cached{0};
    int g = cached.load(std::memory_order_relaxed);
    if (g > 0) return g;
    int dev = 0, cus = 0, per_cu = 0;
    HS_HIP(hipGetDevice(&dev));
    HS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_gemm<T, TM, TN, TK, false>),
                                                        NT, 0));
    g = std::max(1, cus * std::max(1, per_cu));
    cached.store(g, std::memory_order_relaxed);
    return g;
}

template <typename T, int TM, int TN, int TK>
static void launch_shape(const GemmTask* d_tasks, const GemmTerm* d_terms, const GemmTile* d_tiles, int ntiles,
                         bool persistent, hipStream_t s, T* base0, T* base1, int ncols) {
    const int grid = persistent ? std::min(ntiles, resident_grid<T, TM, TN, TK>()) : ntiles;
    if (base0 || base1 || ncols > 0)
        hipLaunchKernelGGL((k_gemm<T, TM, TN, TK, true>), dim3(grid), dim3(NT), 0, s, d_tasks, d_terms, d_tiles,
                           ntiles, base0, base1, ncols);
    else
        hipLaunchKernelGGL((k_gemm<T, TM, TN, TK, false>), dim3(grid), dim3(NT), 0, s, d_tasks, d_terms, d_tiles,
                           ntiles, base0, base1, ncols);
}

template <typename T>
void launch_gemm(const GemmTask* d_tasks, const GemmTerm* d_terms, const GemmTile* d_tiles,
                 int ntiles, double flops, int variant, hipStream_t s, T* base0, T* base1, int ncols,
                 const char* name) {
    if (ntiles <= 0) return;
    ProfScope ps(name ? name : (sizeof(T) == 8 ? "k_gemm" : "k_gemm_f32"), flops, s);
    const bool pers = GEMM_SHAPES[variant].persistent != 0;
    switch (variant) {
        case 1: launch_shape<T, 64, 64, 32>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
        case 2: launch_shape<T, 128, 64, 16>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
        case 3: launch_shape<T, 128, 128, 16>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
        case 4: case 7: launch_shape<T, 32, 32, 64>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
        case 5: launch_shape<T, 32, 32, 128>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
        default: launch_shape<T, 64, 64, 16>(d_tasks, d_terms, d_tiles, ntiles, pers, s, base0, base1, ncols); break;
    }
    check_launch("k_gemm");
}
template void launch_gemm<double>(const GemmTask*, const GemmTerm*, const GemmTile*, int, double, int, hipStream_t,
                                  double*, double*, int, const char*);
template void launch_gemm<float>(const GemmTask*, const GemmTerm*, const GemmTile*, int, double, int, hipStream_t,
                                 float*, float*, int, const char*);

// ---------------------------------------------------------------------------------
// Initial blocks of the first level from the CSR values
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void k_leaf_scatter(const int64_t* row_ptr, const int32_t* col_idx,
                               const double* vals, const int32_t* iperm,
                               const int32_t* pos_super, const int32_t* super_first,
                               void* const* blk_ptr, const int32_t* blk_ld,
                               const int32_t* blk_col, const int32_t* blk_begin, int n) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int pu = iperm[u], su = pos_super[pu], lu = pu - super_first[su];
    for (int64_t t = row_ptr[u]; t < row_ptr[u + 1]; ++t) {
        const int pv = iperm[col_idx[t]], sv = pos_super[pv];
        if (sv < su) continue;
        const int lv = pv - super_first[sv];
        for (int b = blk_begin[su]; b < blk_begin[su + 1]; ++b)
            if (blk_col[b] == sv) {
                static_cast<T*>(blk_ptr[b])[lu + size_t(lv) * blk_ld[b]] = T(vals[t]);
                break;
            }
    }
}

template <typename T>
void launch_leaf_scatter(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                         const int32_t* iperm, const int32_t* pos_super,
                         const int32_t* super_first, void* const* blk_ptr,
                         const int32_t* blk_ld, const int32_t* blk_col,
                         const int32_t* blk_begin, int n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_leaf_scatter<T>, dim3((n + NT - 1) / NT), dim3(NT), 0, s, row_ptr,
                       col_idx, vals, iperm, pos_super, super_first, blk_ptr, blk_ld, blk_col,
                       blk_begin, n);
    check_launch("k_leaf_scatter");
}
template void launch_leaf_scatter<double>(const int64_t*, const int32_t*, const double*, const int32_t*,
                                          const int32_t*, const int32_t*, void* const*, const int32_t*,
                                          const int32_t*, const int32_t*, int, hipStream_t);
template void launch_leaf_scatter<float>(const int64_t*, const int32_t*, const double*, const int32_t*,
                                         const int32_t*, const int32_t*, void* const*, const int32_t*,
                                         const int32_t*, const int32_t*, int, hipStream_t);

// ---------------------------------------------------------------------------------
// Solve phase: forward (gather form) and backward sweeps of one colour
// ---------------------------------------------------------------------------------
// Forward, gather form: V[dst + i] += sign * sum_c G_c(i, :) V[src_c + :]. One workgroup per
// 64 rows of a target; the four waves split the columns of every contribution.
constexpr int FWD_ROWS = WAVE;

template <typename T>
__global__ __launch_bounds__(NT) void k_fwd(const FwdTarget* targets, const FwdContrib* contrib,
                                            T* V, int64_t ldv, int nrhs) {
    const FwdTarget t = targets[blockIdx.y];
    const int r0 = blockIdx.x * FWD_ROWS;
    if (r0 >= t.len) return;
    const int lane = threadIdx.x % WAVE, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int i = r0 + lane;
    __shared__ T part[NT / WAVE][WAVE];
    for (int c = 0; c < nrhs; ++c) {
        T* Vc = V + size_t(c) * ldv;
        T acc[4] = {T(0), T(0), T(0), T(0)};
        if (i < t.len) {
            for (int q = t.c_begin; q < t.c_end; ++q) {
                const FwdContrib f = contrib[q];
                // the source segment (a node of this colour) is not a target of the launch
                const HS_C T* x = cp(Vc + f.src);
                const HS_G T* g = gp(static_cast<const T*>(f.G)) + i;
                int j = wv;
                for (; j + 3 * (NT / WAVE) < f.m; j += 4 * (NT / WAVE)) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int jj = j + u * (NT / WAVE);
                        acc[u] += g[size_t(jj) * f.ldG] * x[jj];
                    }
                }
                for (; j < f.m; j += NT / WAVE) acc[0] += g[size_t(j) * f.ldG] * x[j];
            }
        }
        part[wv][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        __syncthreads();
        if (wv == 0 && i < t.len) {
            T s = T(0);
            for (int w = 0; w < NT / WAVE; ++w) s += part[w][lane];
            Vc[t.dst + i] += T(t.sign) * s;
        }
        __syncthreads();
    }
}

// Several right-hand sides (APPLY_RC per workgroup, blockIdx.z): every factor entry is loaded
// once for all of them; each column is accumulated in exactly the order of k_fwd, so a
// column's result does not depend on the others.
constexpr int APPLY_RC = 8;

template <typename T>
__global__ __launch_bounds__(NT) void k_fwd_m(const FwdTarget* targets, const FwdContrib* contrib,
                                              T* V, int64_t ldv, int nrhs) {
    const FwdTarget t = targets[blockIdx.y];
    const int r0 = blockIdx.x * FWD_ROWS, c0 = blockIdx.z * APPLY_RC;
    if (r0 >= t.len) return;
    const int nc = min(APPLY_RC, nrhs - c0);
    const int lane = threadIdx.x % WAVE, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int i = r0 + lane;
    __shared__ T part[APPLY_RC][NT / WAVE][WAVE];
    T acc[APPLY_RC][4];
#pragma unroll
    for (int c = 0; c < APPLY_RC; ++c)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[c][u] = T(0);
    if (i < t.len) {
        for (int q = t.c_begin; q < t.c_end; ++q) {
            const FwdContrib f = contrib[q];
            // the source segment (a node of this colour) is not a target of the launch
            const HS_C T* x = cp(V + size_t(c0) * ldv + f.src);
            const HS_G T* g = gp(static_cast<const T*>(f.G)) + i;
            int j = wv;
            for (; j + 3 * (NT / WAVE) < f.m; j += 4 * (NT / WAVE)) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jj = j + u * (NT / WAVE);
                    const T gv = g[size_t(jj) * f.ldG];
#pragma unroll
                    for (int c = 0; c < APPLY_RC; ++c)
                        if (c < nc) acc[c][u] += gv * x[size_t(c) * ldv + jj];
                }
            }
            for (; j < f.m; j += NT / WAVE) {
                const T gv = g[size_t(j) * f.ldG];
#pragma unroll
                for (int c = 0; c < APPLY_RC; ++c)
                    if (c < nc) acc[c][0] += gv * x[size_t(c) * ldv + j];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < APPLY_RC; ++c) part[c][wv][lane] = (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
    __syncthreads();
    if (wv == 0 && i < t.len) {
        for (int c = 0; c < nc; ++c) {
            T s = T(0);
            for (int w = 0; w < NT / WAVE; ++w) s += part[c][w][lane];
            V[size_t(c0 + c) * ldv + t.dst + i] += T(t.sign) * s;
        }
    }
}

template <typename T>
void launch_fwd(const FwdTarget* t, const FwdContrib* c, int nt, int max_len, T* V, int64_t ldv,
                int nrhs, double bytes, hipStream_t s) {
    if (nt <= 0 || max_len <= 0) return;
    ProfScope ps(sizeof(T) == 8 ? "k_fwd" : "k_fwd_f32", bytes, s);
    if (nrhs == 1) {
        hipLaunchKernelGGL(k_fwd<T>, dim3((max_len + FWD_ROWS - 1) / FWD_ROWS, nt), dim3(NT), 0, s, t, c, V,
                           ldv, nrhs);
        check_launch("k_fwd");
    } else {
        hipLaunchKernelGGL(k_fwd_m<T>, dim3((max_len + FWD_ROWS - 1) / FWD_ROWS, nt, (nrhs + APPLY_RC - 1) / APPLY_RC),
                           dim3(NT), 0, s, t, c, V, ldv, nrhs);
        check_launch("k_fwd_m");
    }
}
template void launch_fwd<double>(const FwdTarget*, const FwdContrib*, int, int, double*, int64_t, int, double,
                                 hipStream_t);
template void launch_fwd<float>(const FwdTarget*, const FwdContrib*, int, int, float*, int64_t, int, double,
                                hipStream_t);

// Backward: x_s = Gm^T v with v = [phi_s; -x_N; x_r] gathered into LDS (phi from V, the
// solutions from X), written to X. Each workgroup takes BWD_COLS columns of one node (two
// per wave); every column is a wave-wide dot product with eight loads in flight per lane.
constexpr int BWD_MAX_ROWS = 6144;
constexpr int BWD_COLS = 8;

template <typename T>
__global__ __launch_bounds__(NT) void k_bwd(const BwdNode* nodes, const BwdSeg* segs, const T* V,
                                            T* X, int64_t ldv, int nrhs) {
    const BwdNode nd = nodes[blockIdx.y];
    const int j0 = blockIdx.x * BWD_COLS;
    if (j0 >= nd.m) return;
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    __shared__ T v[BWD_MAX_ROWS];
    for (int c = 0; c < nrhs; ++c) {
        const T* Vc = V + size_t(c) * ldv;
        T* Xc = X + size_t(c) * ldv;
        int pos = 0;
        for (int q = nd.seg_begin; q < nd.seg_end; ++q) {
            const BwdSeg sg = segs[q];
            const T* src = (sg.buf ? Xc : Vc) + sg.off;
            for (int i = threadIdx.x; i < sg.len; i += NT) v[pos + i] = T(sg.sign) * src[i];
            pos += sg.len;
        }
        __syncthreads();
        for (int jj = wv; jj < BWD_COLS; jj += NT / WAVE) {
            const int j = j0 + jj;
            if (j >= nd.m) break;
            const HS_G T* g = gp(static_cast<const T*>(nd.G)) + size_t(j) * nd.ldG;
            T a[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
            int i = lane;
            for (; i + 7 * WAVE < nd.rows; i += 8 * WAVE) {
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] += g[i + u * WAVE] * v[i + u * WAVE];
            }
            for (; i < nd.rows; i += WAVE) a[0] += g[i] * v[i];
            const T acc = wave_sum(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])));
            if (lane == 0) Xc[nd.dst + j] = acc;
        }
        __syncthreads();
    }
}

// Several right-hand sides (APPLY_RC per workgroup, blockIdx.z): v is gathered BWD_CHUNK rows
// at a time for all of them, each factor entry is loaded once; a column's sums follow the
// order of k_bwd exactly (rows lane + 64 u + 512 t in a[u] while all eight exist, the
// lane's remaining rows in a[0]).
constexpr int BWD_CHUNK = 512;

template <typename T>
__global__ __launch_bounds__(NT) void k_bwd_m(const BwdNode* nodes, const BwdSeg* segs, const T* V,
                                              T* X, int64_t ldv, int nrhs) {
    const BwdNode nd = nodes[blockIdx.y];
    const int j0 = blockIdx.x * BWD_COLS, c0 = blockIdx.z * APPLY_RC;
    if (j0 >= nd.m) return;
    const int nc = min(APPLY_RC, nrhs - c0);
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    __shared__ T v[APPLY_RC][BWD_CHUNK];
    constexpr int JW = BWD_COLS / (NT / WAVE);           // output columns per wave
    T a[JW][APPLY_RC][8];
#pragma unroll
    for (int q = 0; q < JW; ++q)
#pragma unroll
        for (int c = 0; c < APPLY_RC; ++c)
#pragma unroll
            for (int u = 0; u < 8; ++u) a[q][c][u] = T(0);
    for (int r0 = 0; r0 < nd.rows; r0 += BWD_CHUNK) {
        const int r1 = min(nd.rows, r0 + BWD_CHUNK);
        __syncthreads();
        int pos = 0;
        for (int q = nd.seg_begin; q < nd.seg_end; ++q) {
            const BwdSeg sg = segs[q];
            const int lo = max(pos, r0), hi = min(pos + sg.len, r1);
            for (int e = threadIdx.x; e < APPLY_RC * (hi - lo); e += NT) {
                const int c = e / (hi - lo), r = lo + e % (hi - lo);
                if (c < nc) {
                    const T* src = (sg.buf ? X : V) + size_t(c0 + c) * ldv + sg.off;
                    v[c][r - r0] = T(sg.sign) * src[r - pos];
                }
            }
            pos += sg.len;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < JW; ++q) {
            const int j = j0 + wv + q * (NT / WAVE);
            if (j >= nd.m) break;
            const HS_G T* g = gp(static_cast<const T*>(nd.G)) + size_t(j) * nd.ldG;
            if (r0 + lane + 7 * WAVE < nd.rows) {           // this lane's rows of the block all exist
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = r0 + lane + u * WAVE;
                    const T gv = g[i];
#pragma unroll
                    for (int c = 0; c < APPLY_RC; ++c)
                        if (c < nc) a[q][c][u] += gv * v[c][i - r0];
                }
            } else {                                        // the rest, in a[0] (as k_bwd)
                for (int i = r0 + lane; i < r1; i += WAVE) {
                    const T gv = g[i];
#pragma unroll
                    for (int c = 0; c < APPLY_RC; ++c)
                        if (c < nc) a[q][c][0] += gv * v[c][i - r0];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < JW; ++q) {
        const int j = j0 + wv + q * (NT / WAVE);
#pragma unroll
        for (int c = 0; c < APPLY_RC; ++c) {
            const T acc = wave_sum(((a[q][c][0] + a[q][c][1]) + (a[q][c][2] + a[q][c][3])) +
                                        ((a[q][c][4] + a[q][c][5]) + (a[q][c][6] + a[q][c][7])));
            if (lane == 0 && j < nd.m && c < nc) X[size_t(c0 + c) * ldv + nd.dst + j] = acc;
        }
    }
}

template <typename T>
void launch_bwd(const BwdNode* nodes, const BwdSeg* segs, int nn, int max_m, const T* V, T* X,
                int64_t ldv, int nrhs, double bytes, hipStream_t s) {
    if (nn <= 0 || max_m <= 0) return;
    ProfScope ps(sizeof(T) == 8 ? "k_bwd" : "k_bwd_f32", bytes, s);
    if (nrhs == 1) {
        hipLaunchKernelGGL(k_bwd<T>, dim3((max_m + BWD_COLS - 1) / BWD_COLS, nn), dim3(NT), 0, s, nodes, segs,
                           V, X, ldv, nrhs);
        check_launch("k_bwd");
    } else {
        hipLaunchKernelGGL(k_bwd_m<T>, dim3((max_m + BWD_COLS - 1) / BWD_COLS, nn, (nrhs + APPLY_RC - 1) / APPLY_RC),
                           dim3(NT), 0, s, nodes, segs, V, X, ldv, nrhs);
        check_launch("k_bwd_m");
    }
}
template void launch_bwd<double>(const BwdNode*, const BwdSeg*, int, int, const double*, double*, int64_t, int,
                                 double, hipStream_t);
template void launch_bwd<float>(const BwdNode*, const BwdSeg*, int, int, const float*, float*, int64_t, int,
                                double, hipStream_t);

// ---------------------------------------------------------------------------------
// Permutations, SpMV, BLAS-1
// ---------------------------------------------------------------------------------
// dst[p] = src[perm[p]] (into the solve vector, in its storage type)
template <typename T>
__global__ void k_gather_perm(const double* src, int lds, T* dst, int64_t ldd,
                              const int32_t* perm, int n, int nrhs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    for (int c = 0; c < nrhs; ++c) dst[p + c * ldd] = T(src[u + size_t(c) * lds]);
}

template <typename T>
void launch_gather_perm(const double* src, int lds, T* dst, int64_t ldd, const int32_t* perm,
                        int n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_perm<T>, dim3((n + NT - 1) / NT), dim3(NT), 0, s, src, lds, dst,
                       ldd, perm, n, nrhs);
    check_launch("k_gather_perm");
}
template void launch_gather_perm<double>(const double*, int, double*, int64_t, const int32_t*, int, int,
                                         hipStream_t);
template void launch_gather_perm<float>(const double*, int, float*, int64_t, const int32_t*, int, int,
                                        hipStream_t);

// dst[perm[p]] = src[p] (out of the solve vector, widened to double)
template <typename T>
__global__ void k_scatter_perm(const T* src, int64_t lds, double* dst, int ldd,
                               const int32_t* perm, int n, int nrhs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    for (int c = 0; c < nrhs; ++c) dst[u + size_t(c) * ldd] = double(src[p + c * lds]);
}

template <typename T>
void launch_scatter_perm(const T* src, int64_t lds, double* dst, int ldd,
                         const int32_t* perm, int n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_perm<T>, dim3((n + NT - 1) / NT), dim3(NT), 0, s, src, lds, dst,
                       ldd, perm, n, nrhs);
    check_launch("k_scatter_perm");
}
template void launch_scatter_perm<double>(const double*, int64_t, double*, int, const int32_t*, int, int,
                                          hipStream_t);
template void launch_scatter_perm<float>(const float*, int64_t, double*, int, const int32_t*, int, int,
                                         hipStream_t);

// Rounds factor blocks to single precision for the FP32 solve phase: one task per block
// (blockIdx.y), round to nearest.
__global__ __launch_bounds__(NT) void k_demote(const DemoteTask* tasks) {
    const DemoteTask t = tasks[blockIdx.y];
    for (int64_t i = blockIdx.x * int64_t(NT) + threadIdx.x; i < t.count; i += int64_t(gridDim.x) * NT)
        t.dst[i] = float(t.src[i]);
}

void launch_demote(const DemoteTask* d_tasks, int ntasks, double elems, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_demote", 12.0 * elems, s);
    hipLaunchKernelGGL(k_demote, dim3(64, ntasks), dim3(NT), 0, s, d_tasks);
    check_launch("k_demote");
}

__global__ void k_spmv(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                       const double* x, double* y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) acc += vals[t] * x[col_idx[t]];
    y[i] = acc;
}

void launch_spmv(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                 const double* x, double* y, int n, int64_t nnz, hipStream_t s) {
    // values + column indices + row pointers + x once + y once
    ProfScope ps("k_spmv", 12.0 * nnz + 8.0 * (n + 1) + 16.0 * n, s);
    hipLaunchKernelGGL(k_spmv, dim3((n + NT - 1) / NT), dim3(NT), 0, s, row_ptr, col_idx, vals,
                       x, y, n);
    check_launch("k_spmv");
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + NT - 1) / NT;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3(unsigned(nb)), dim3(NT), 0, s, p, v, n);
    check_launch("k_fill");
}
template void launch_fill<double>(double*, double, int64_t, hipStream_t);
template void launch_fill<float>(float*, float, int64_t, hipStream_t);
template void launch_fill<int>(int*, int, int64_t, hipStream_t);

// flag = 1 when some v[i] is NaN or infinite (flag starts at 0; racing writers store the
// same value)
__global__ void k_nonfinite(const double* v, int64_t n, int* flag) {
    bool bad = false;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        bad |= !isfinite(v[i]);
    if (bad) *flag = 1;
}

void launch_check_finite(const double* v, int64_t n, int* flag, hipStream_t s) {
    launch_fill<int>(flag, 0, 1, s);
    if (n <= 0) return;
    int64_t nb = (n + NT - 1) / NT;
    if (nb > 2048) nb = 2048;
    hipLaunchKernelGGL(k_nonfinite, dim3(unsigned(nb)), dim3(NT), 0, s, v, n, flag);
    check_launch("k_nonfinite");
}

}  // namespace hs
