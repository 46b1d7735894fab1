// HIP kernels for gfx950 (wave64). FP64 throughout.
//
//  k_copy        batched 2-D block copies (optional transpose)          block gather / merge
//  k_gemm        grouped GEMM over tile lists, C = bC + a sum op(A)op(B) Gram, Schur, T_N, L_nr, R
//  k_chol_inv    per-block Cholesky + explicit inverse                  pivot A_ss^-1, S^-1
//  k_compress    per-node eigen-decomposition of the Gram matrix of the well-separated block
//                (Householder tridiagonalisation, implicit QL with shifts, parallel Sturm
//                bisection), GC basis split, truncation                 compression
//  k_fwd / k_bwd level sweeps of the solve phase                        apply
//  k_spmv, k_dot*, k_axpy2, k_xpby, gathers/scatters                    outer PCG
#include <cfloat>

#include "hs_internal.h"

namespace hs {

constexpr int NT = 256;          // threads per workgroup (4 waves)

static void check_launch(const char* name) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw Error{HSOLVE_ERR_DEVICE, std::string("launch of ") + name + ": " + hipGetErrorString(e)};
}
constexpr int WAVE = 64;

__device__ inline double wave_sum(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// block-wide sum; `red` must hold NT/WAVE doubles; result valid in every thread
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / WAVE; ++i) s += red[i];
    return s;
}

// ---------------------------------------------------------------------------------
// Copies
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_copy(const CopyTask* tasks) {
    const CopyTask t = tasks[blockIdx.x];
    __shared__ double tile[32][33];
    if (!t.trans) {
        for (int j = 0; j < t.cols; ++j)
            for (int i = threadIdx.x; i < t.rows; i += NT)
                t.dst[i + size_t(j) * t.ldd] = t.src[i + size_t(j) * t.lds];
        return;
    }
    // dst(i,j) = src(j,i), through 32x32 tiles
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;   // 32 x 8
    for (int i0 = 0; i0 < t.rows; i0 += 32)
        for (int j0 = 0; j0 < t.cols; j0 += 32) {
            for (int r = ty; r < 32; r += 8) {           // read src rows j0+r? src is cols x rows
                int si = j0 + tx, sj = i0 + r;               // src(si, sj)
                if (si < t.cols && sj < t.rows) tile[r][tx] = t.src[si + size_t(sj) * t.lds];
            }
            __syncthreads();
            for (int r = ty; r < 32; r += 8) {
                int di = i0 + tx, dj = j0 + r;               // dst(di, dj) = src(dj, di)
                if (di < t.rows && dj < t.cols) t.dst[di + size_t(dj) * t.ldd] = tile[tx][r];
            }
            __syncthreads();
        }
}

void launch_copy(const CopyTask* d_tasks, int ntasks, double bytes, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_copy", bytes, s);
    hipLaunchKernelGGL(k_copy, dim3(ntasks), dim3(NT), 0, s, d_tasks);
    check_launch("k_copy");
}

// ---------------------------------------------------------------------------------
// Grouped GEMM: 64 x 64 output tiles, 256 threads, 4 x 4 outputs per thread
// ---------------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 16;

__global__ __launch_bounds__(NT) void k_gemm(const GemmTask* tasks, const GemmTerm* terms,
                                             const GemmTile* tiles) {
    const GemmTile tl = tiles[blockIdx.x];
    const GemmTask T = tasks[tl.task];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    __shared__ double As[TK][TM + 1];
    __shared__ double Bs[TK][TN + 1];
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    const int i0 = tl.ti * TM, j0 = tl.tj * TN;
    for (int t = T.t_begin; t < T.t_end; ++t) {
        const GemmTerm g = terms[t];
        for (int k0 = 0; k0 < g.K; k0 += TK) {
            for (int e = tid; e < TM * TK; e += NT) {
                int ii, kk;
                if (!g.transA) { ii = e % TM; kk = e / TM; } else { kk = e % TK; ii = e / TK; }
                const int gi = i0 + ii, gk = k0 + kk;
                double v = 0.0;
                if (gi < T.M && gk < g.K)
                    v = g.transA ? g.A[gk + size_t(gi) * g.lda] : g.A[gi + size_t(gk) * g.lda];
                As[kk][ii] = v;
            }
            for (int e = tid; e < TN * TK; e += NT) {
                int jj, kk;
                if (g.transB) { jj = e % TN; kk = e / TN; } else { kk = e % TK; jj = e / TK; }
                const int gj = j0 + jj, gk = k0 + kk;
                double v = 0.0;
                if (gj < T.N && gk < g.K)
                    v = g.transB ? g.B[gj + size_t(gk) * g.ldb] : g.B[gk + size_t(gj) * g.ldb];
                Bs[kk][jj] = v;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < TK; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int x = 0; x < 4; ++x) a[x] = As[kk][tx + 16 * x];
#pragma unroll
                for (int y = 0; y < 4; ++y) b[y] = Bs[kk][ty + 16 * y];
#pragma unroll
                for (int x = 0; x < 4; ++x)
#pragma unroll
                    for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int i = i0 + tx + 16 * x, j = j0 + ty + 16 * y;
            if (i < T.M && j < T.N) {
                double* c = T.C + i + size_t(j) * T.ldc;
                const double old = (T.beta == 0.0) ? 0.0 : T.beta * (*c);
                *c = old + T.alpha * acc[x][y];
            }
        }
}

void launch_gemm(const GemmTask* d_tasks, const GemmTerm* d_terms, const GemmTile* d_tiles,
                 int ntiles, double flops, hipStream_t s) {
    if (ntiles <= 0) return;
    ProfScope ps("k_gemm", flops, s);
    hipLaunchKernelGGL(k_gemm, dim3(ntiles), dim3(NT), 0, s, d_tasks, d_terms, d_tiles);
    check_launch("k_gemm");
}

// ---------------------------------------------------------------------------------
// Cholesky A = L L^T (lower, in place) and explicit A^{-1} = L^{-T} L^{-1}
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_chol_inv(const CholTask* tasks, int* fail) {
    const CholTask T = tasks[blockIdx.x];
    const int m = T.m, lda = T.lda, tid = threadIdx.x;
    double* A = T.A;
    __shared__ int bad;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            const double djj = A[j + size_t(j) * lda];
            if (!(djj > 0.0) || !isfinite(djj)) bad = 1;
            else A[j + size_t(j) * lda] = sqrt(djj);
        }
        __syncthreads();
        if (bad) break;
        const double piv = A[j + size_t(j) * lda];
        for (int i = j + 1 + tid; i < m; i += NT) A[i + size_t(j) * lda] /= piv;
        __syncthreads();
        for (int k = j + 1; k < m; ++k) {
            const double akj = A[k + size_t(j) * lda];
            for (int i = k + tid; i < m; i += NT)
                A[i + size_t(k) * lda] -= A[i + size_t(j) * lda] * akj;
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) fail[T.id] = 1;
        return;
    }
    // column c of A^{-1}: L y = e_c, then L^T x = y (in place in Ainv[:, c])
    for (int c = tid; c < m; c += NT) {
        double* x = T.Ainv + size_t(c) * T.ldi;
        for (int i = 0; i < c; ++i) x[i] = 0.0;
        for (int i = c; i < m; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int j = c; j < i; ++j) s -= A[i + size_t(j) * lda] * x[j];
            x[i] = s / A[i + size_t(i) * lda];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = x[i];
            for (int j = i + 1; j < m; ++j) s -= A[j + size_t(i) * lda] * x[j];
            x[i] = s / A[i + size_t(i) * lda];
        }
    }
}

void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops,
                     hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_chol_inv", flops, s);
    hipLaunchKernelGGL(k_chol_inv, dim3(ntasks), dim3(NT), 0, s, d_tasks, d_fail);
    check_launch("k_chol_inv");
}

// ---------------------------------------------------------------------------------
// Compression: eigen-decomposition of the Gram matrix G = A_sw A_sw^T
// ---------------------------------------------------------------------------------
constexpr int MAXN = 1024;       // largest super node handled by k_compress

struct EigShared {
    double d[MAXN], e[MAXN], tau[MAXN], v[MAXN], w[MAXN], rc[MAXN], rs[MAXN];
    int idx[MAXN];
    double red[NT / WAVE];
    double scal[4];
    int iscal[4];
    int pts[NT + 1];
};

// Householder tridiagonalisation of the symmetric nn x nn matrix H (column-major, ld),
// Q^T H Q = T. Reflector j acts on rows j+1.., its vector (v[0] = 1 implicit) is kept in
// H(j+2.., j) and tau[j]; the diagonal goes to d, the sub-diagonal to e.
__device__ void tridiagonalize(double* H, int ld, int nn, EigShared& S) {
    const int tid = threadIdx.x;
    for (int j = 0; j + 2 < nn; ++j) {
        double* col = H + size_t(j) * ld;
        double part = 0.0;
        for (int i = j + 2 + tid; i < nn; i += NT) part += col[i] * col[i];
        const double xn2 = block_sum(part, S.red);
        const double alpha = col[j + 1];
        double tau = 0.0, beta = alpha;
        if (xn2 > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tau = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
            for (int i = j + 2 + tid; i < nn; i += NT) col[i] *= scal;
        }
        __syncthreads();
        const int len = nn - j - 1;                       // trailing block rows j+1..nn-1
        for (int i = tid; i < len; i += NT) S.v[i] = (i == 0) ? 1.0 : (xn2 > 0.0 ? col[j + 1 + i] : 0.0);
        if (tid == 0) { S.tau[j] = tau; S.e[j] = beta; }
        __syncthreads();
        if (tau != 0.0) {
            double* T22 = H + size_t(j + 1) * ld + (j + 1);
            double pv_part = 0.0;
            for (int i = tid; i < len; i += NT) {
                double acc = 0.0;
                for (int l = 0; l < len; ++l) acc += T22[i + size_t(l) * ld] * S.v[l];
                acc *= tau;
                S.w[i] = acc;
                pv_part += acc * S.v[i];
            }
            const double K = 0.5 * tau * block_sum(pv_part, S.red);
            for (int i = tid; i < len; i += NT) S.w[i] -= K * S.v[i];
            __syncthreads();
            for (int l = 0; l < len; ++l) {
                const double vl = S.v[l], wl = S.w[l];
                for (int i = tid; i < len; i += NT)
                    T22[i + size_t(l) * ld] -= S.v[i] * wl + S.w[i] * vl;
            }
            __syncthreads();
        }
    }
    for (int j = tid; j < nn; j += NT) S.d[j] = H[j + size_t(j) * ld];
    if (tid == 0) {
        if (nn >= 2) S.e[nn - 2] = H[(nn - 1) + size_t(nn - 2) * ld];
        S.e[nn - 1] = 0.0;
        if (nn >= 2) S.tau[nn - 2] = 0.0;
        S.tau[nn - 1] = 0.0;
    }
    __syncthreads();
}

// x <- Q x for a vector stored at x (length nn) using the reflectors left in H; executed by
// one wave (lane-parallel).
__device__ void backtransform_wave(const double* H, int ld, int nn, const double* tau, double* x) {
    const int lane = threadIdx.x % WAVE;
    for (int j = nn - 3; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        const double* col = H + size_t(j) * ld;
        double part = 0.0;
        for (int i = j + 1 + lane; i < nn; i += WAVE) {
            const double vi = (i == j + 1) ? 1.0 : col[i];
            part += vi * x[i];
        }
        const double dot = wave_sum(part) * tj;
        for (int i = j + 1 + lane; i < nn; i += WAVE) {
            const double vi = (i == j + 1) ? 1.0 : col[i];
            x[i] -= dot * vi;
        }
    }
}

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

// largest eigenvalue of the tridiagonal (S.d, S.e) by parallel multisection
__device__ double largest_eigenvalue(int nn, EigShared& S) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        double lo = S.d[0], hi = S.d[0], me = 0.0;
        for (int i = 0; i < nn; ++i) {
            const double r = (i > 0 ? fabs(S.e[i - 1]) : 0.0) + (i + 1 < nn ? fabs(S.e[i]) : 0.0);
            lo = fmin(lo, S.d[i] - r);
            hi = fmax(hi, S.d[i] + r);
            if (i + 1 < nn) me = fmax(me, S.e[i] * S.e[i]);
        }
        const double pad = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 1e-300;
        S.scal[0] = lo - pad;
        S.scal[1] = hi + pad;
        S.scal[2] = fmax(1e-300, 1e-300 * me);
    }
    __syncthreads();
    for (int round = 0; round < 10; ++round) {
        const double lo = S.scal[0], hi = S.scal[1], pivmin = S.scal[2];
        __syncthreads();
        const double x = lo + (hi - lo) * double(tid + 1) / double(NT + 1);
        S.pts[tid] = sturm_count(S.d, S.e, nn, x, pivmin) == nn ? 1 : 0;
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            while (t < NT && !S.pts[t]) ++t;
            const double xl = (t == 0) ? lo : lo + (hi - lo) * double(t) / double(NT + 1);
            const double xh = (t == NT) ? hi : lo + (hi - lo) * double(t + 1) / double(NT + 1);
            S.scal[0] = xl;
            S.scal[1] = xh;
        }
        __syncthreads();
    }
    return 0.5 * (S.scal[0] + S.scal[1]);
}

// Implicit QL with shifts on (S.d, S.e) (nn x nn); Z (column-major, ld) starts as the
// identity and ends with the eigenvectors of the tridiagonal in its columns.
// Returns false if an eigenvalue fails to converge.
__device__ bool ql_implicit(int nn, double* Z, int ldz, EigShared& S) {
    const int tid = threadIdx.x;
    for (int c = 0; c < nn; ++c)
        for (int i = tid; i < nn; i += NT) Z[i + size_t(c) * ldz] = (i == c) ? 1.0 : 0.0;
    // Deflate against the norm of the whole tridiagonal (eigenvalues are needed to an
    // absolute accuracy relative to the largest one): clusters of numerically zero
    // eigenvalues then split at once instead of iterating on rounding noise.
    if (tid == 0) {
        double tn = 0.0;
        for (int i = 0; i < nn; ++i) tn = fmax(tn, fabs(S.d[i]) + fabs(S.e[i]));
        S.scal[3] = tn;
    }
    __syncthreads();
    const double tnorm = S.scal[3];
    for (int l = 0; l < nn; ++l) {
        for (int iter = 0;; ++iter) {
            // S.iscal: [0] = m (deflation point), [1] = lowest rotation index, [2] = status
            if (tid == 0) {
                int m = l;
                for (; m < nn - 1; ++m)
                    if (fabs(S.e[m]) <= DBL_EPSILON * tnorm) break;
                S.iscal[0] = m;
                S.iscal[2] = 0;
                if (m != l) {
                    if (iter >= 80) {
                        S.iscal[2] = 2;
                    } else {
                        double g = (S.d[l + 1] - S.d[l]) / (2.0 * S.e[l]);
                        double r = hypot(g, 1.0);
                        g = S.d[m] - S.d[l] + S.e[l] / (g + copysign(r, g));
                        double s = 1.0, c = 1.0, p = 0.0;
                        int i = m - 1;
                        bool under = false;
                        for (; i >= l; --i) {
                            const double f = s * S.e[i], b = c * S.e[i];
                            r = hypot(f, g);
                            S.e[i + 1] = r;
                            if (r == 0.0) {
                                S.d[i + 1] -= p;
                                S.e[m] = 0.0;
                                under = true;
                                break;
                            }
                            s = f / r;
                            c = g / r;
                            g = S.d[i + 1] - p;
                            r = (S.d[i] - g) * s + 2.0 * c * b;
                            p = s * r;
                            S.d[i + 1] = g + p;
                            g = c * r - b;
                            S.rc[i] = c;
                            S.rs[i] = s;
                        }
                        S.iscal[1] = under ? i + 1 : l;
                        if (!under) {
                            S.d[l] -= p;
                            S.e[l] = g;
                            S.e[m] = 0.0;
                        }
                        S.iscal[2] = 1;
                    }
                }
            }
            __syncthreads();
            const int m = S.iscal[0], status = S.iscal[2], lo = S.iscal[1];
            if (status == 2) return false;
            if (status == 0) break;
            // rotations i = m-1 .. lo act on columns (i, i+1) of Z
            for (int k = tid; k < nn; k += NT) {
                double zi1 = Z[k + size_t(m) * ldz];
                for (int i = m - 1; i >= lo; --i) {
                    const double zi = Z[k + size_t(i) * ldz];
                    Z[k + size_t(i + 1) * ldz] = S.rs[i] * zi + S.rc[i] * zi1;
                    zi1 = S.rc[i] * zi - S.rs[i] * zi1;
                }
                Z[k + size_t(lo) * ldz] = zi1;
            }
            __syncthreads();
        }
    }
    return true;
}

// Two-sided application of the reflector I - tau v v^T (v nonzero on rows >= r0) to the
// symmetric m x m matrix H.
__device__ void reflect_two_sided(double* H, int ld, int m, const double* v, double tau,
                                  EigShared& S) {
    const int tid = threadIdx.x;
    double pv_part = 0.0;
    for (int i = tid; i < m; i += NT) {
        double acc = 0.0;
        for (int l = 0; l < m; ++l) acc += H[i + size_t(l) * ld] * v[l];
        acc *= tau;
        S.w[i] = acc;
        pv_part += acc * v[i];
    }
    const double K = 0.5 * tau * block_sum(pv_part, S.red);
    for (int i = tid; i < m; i += NT) S.w[i] -= K * v[i];
    __syncthreads();
    for (int l = 0; l < m; ++l) {
        const double vl = v[l], wl = S.w[l];
        if (vl == 0.0 && wl == 0.0) continue;
        for (int i = tid; i < m; i += NT) H[i + size_t(l) * ld] -= v[i] * wl + S.w[i] * vl;
    }
    __syncthreads();
}

__global__ __launch_bounds__(NT) void k_compress(const CompressTask* tasks, int variant,
                                                 double eps, int* rank) {
    extern __shared__ char smem_raw[];
    EigShared& S = *reinterpret_cast<EigShared*>(smem_raw);
    const CompressTask T = tasks[blockIdx.x];
    const int m = T.m, tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
    double* H = T.work;                            // m x m
    double* Zq = T.work + size_t(m) * m;           // m x m eigenvectors
    double* gcv = T.work + size_t(2) * m * m;      // GC reflectors: up to 16 vectors of m
    double* gct = gcv + size_t(16) * m;            // their tau
    double* U = T.U;

    // scale G by its largest entry (eigenvectors unchanged, decisions are relative)
    double gmax = 0.0;
    for (size_t i = tid; i < size_t(m) * m; i += NT) gmax = fmax(gmax, fabs(T.G[i]));
    for (int o = WAVE / 2; o > 0; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o, WAVE));
    if (lane == 0) S.red[wv] = gmax;
    __syncthreads();
    gmax = fmax(fmax(S.red[0], S.red[1]), fmax(S.red[2], S.red[3]));
    __syncthreads();
    const double gscale = (gmax > 0.0 && isfinite(gmax)) ? 1.0 / gmax : 1.0;
    for (size_t i = tid; i < size_t(m) * m; i += NT) H[i] = T.G[i] * gscale;
    __syncthreads();

    int q = 0;
    double lam_max;
    if (variant == HSOLVE_LORASP) {
        tridiagonalize(H, m, m, S);
        if (!ql_implicit(m, Zq, m, S)) { if (tid == 0) rank[T.id] = -1; return; }
        double mx = -DBL_MAX;
        for (int i = 0; i < m; ++i) mx = fmax(mx, S.d[i]);
        lam_max = mx;
    } else {
        tridiagonalize(H, m, m, S);
        lam_max = largest_eigenvalue(m, S);
        // U1 = orthonormal basis of the columns of Z (modified Gram-Schmidt, twice)
        for (int c = 0; c < T.nz && q < m; ++c) {
            const double* z = T.Z + size_t(c) * m;
            double* u = U + size_t(q) * m;
            double part = 0.0;
            for (int i = tid; i < m; i += NT) { u[i] = z[i]; part += z[i] * z[i]; }
            const double nz = sqrt(block_sum(part, S.red));
            if (nz == 0.0) continue;
            for (int pass = 0; pass < 2; ++pass)
                for (int b = 0; b < q; ++b) {
                    const double* ub = U + size_t(b) * m;
                    double pp = 0.0;
                    for (int i = tid; i < m; i += NT) pp += ub[i] * u[i];
                    const double dot = block_sum(pp, S.red);
                    for (int i = tid; i < m; i += NT) u[i] -= dot * ub[i];
                    __syncthreads();
                }
            part = 0.0;
            for (int i = tid; i < m; i += NT) part += u[i] * u[i];
            const double nu = sqrt(block_sum(part, S.red));
            if (nu > 1e-10 * nz) {
                for (int i = tid; i < m; i += NT) u[i] /= nu;
                __syncthreads();
                ++q;
            }
        }
        // Householder reflectors W = H_{q-1}..H_0 with W U1 = [R; 0]; the complement of U1
        // is W^T [0; I]. Project G there: G' = (W G W^T)(q:, q:)
        for (size_t i = tid; i < size_t(m) * m; i += NT) H[i] = T.G[i] * gscale;
        for (int t = 0; t < q; ++t) {
            // x = (H_{t-1}..H_0 u_t)(t..m-1); stored temporarily in Zq column 0
            double* x = Zq;
            for (int i = tid; i < m; i += NT) x[i] = U[i + size_t(t) * m];
            __syncthreads();
            for (int b = 0; b < t; ++b) {
                const double* vb = gcv + size_t(b) * m;
                double pp = 0.0;
                for (int i = tid; i < m; i += NT) pp += vb[i] * x[i];
                const double dot = block_sum(pp, S.red) * gct[b];
                for (int i = tid; i < m; i += NT) x[i] -= dot * vb[i];
                __syncthreads();
            }
            double part = 0.0;
            for (int i = t + 1 + tid; i < m; i += NT) part += x[i] * x[i];
            const double xn2 = block_sum(part, S.red);
            const double alpha = x[t];
            double* vt = gcv + size_t(t) * m;
            double tau = 0.0;
            if (xn2 > 0.0) {
                const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
                tau = (beta - alpha) / beta;
                const double scal = 1.0 / (alpha - beta);
                for (int i = tid; i < m; i += NT)
                    vt[i] = (i < t) ? 0.0 : (i == t ? 1.0 : x[i] * scal);
            } else {
                for (int i = tid; i < m; i += NT) vt[i] = (i == t) ? 1.0 : 0.0;
            }
            if (tid == 0) gct[t] = tau;
            __syncthreads();
            if (tau != 0.0) reflect_two_sided(H, m, m, vt, tau, S);
        }
        const int nn = m - q;
        if (nn > 0) {
            tridiagonalize(H + size_t(q) * m + q, m, nn, S);
            if (!ql_implicit(nn, Zq, nn, S)) { if (tid == 0) rank[T.id] = -1; return; }
        }
    }
    const int nn = m - q;
    // select the leading eigenvalues of the (projected) Gram matrix
    const int cap = min(nn, T.wt);
    const double thr = eps * eps * fmax(lam_max, 0.0);   // zero G: nothing passes
    // descending order (NaN last), ties by index: a permutation whatever the values
    for (int j = tid; j < nn; j += NT) {
        int r = 0;
        const double dj = isnan(S.d[j]) ? -DBL_MAX : S.d[j];
        for (int i = 0; i < nn; ++i) {
            const double di = isnan(S.d[i]) ? -DBL_MAX : S.d[i];
            r += (di > dj) || (di == dj && i < j);
        }
        S.idx[r] = j;
    }
    __syncthreads();
    if (tid == 0) {
        int k2 = 0;
        if (eps == 0.0) k2 = cap;
        else while (k2 < cap && S.d[S.idx[k2]] > thr) ++k2;
        if (q + k2 == 0 && cap > 0) k2 = 1;
        S.iscal[3] = k2;
    }
    __syncthreads();
    const int k2 = S.iscal[3];
    // eigenvectors of the selected eigenvalues, back in the m-dim coordinates
    const double* Hs = (variant == HSOLVE_LORASP) ? H : H + size_t(q) * m + q;
    for (int r = wv; r < k2; r += NT / WAVE) {
        double* u = U + size_t(q + r) * m;
        const double* z = Zq + size_t(S.idx[r]) * nn;
        for (int i = lane; i < m; i += WAVE) u[i] = (i < q) ? 0.0 : z[i - q];
        backtransform_wave(Hs, m, nn, S.tau, u + q);
        for (int t = q - 1; t >= 0; --t) {       // u <- H_0 .. H_{q-1} u
            const double* vt = gcv + size_t(t) * m;
            const double tt = gct[t];
            if (tt == 0.0) continue;
            double part = 0.0;
            for (int i = lane; i < m; i += WAVE) part += vt[i] * u[i];
            const double dot = wave_sum(part) * tt;
            for (int i = lane; i < m; i += WAVE) u[i] -= dot * vt[i];
        }
    }
    if (tid == 0) rank[T.id] = q + k2;
}

void launch_compress(const CompressTask* d_tasks, int ntasks, int variant, double eps,
                     int* d_rank, double flops, hipStream_t s) {
    if (ntasks <= 0) return;
    ProfScope ps("k_compress", flops, s);
    hipLaunchKernelGGL(k_compress, dim3(ntasks), dim3(NT), sizeof(EigShared), s, d_tasks,
                       variant, eps, d_rank);
    check_launch("k_compress");
}

// ---------------------------------------------------------------------------------
// Initial blocks of the first level from the CSR values
// ---------------------------------------------------------------------------------
__global__ void k_leaf_scatter(const int64_t* row_ptr, const int32_t* col_idx,
                               const double* vals, const int32_t* iperm,
                               const int32_t* pos_super, const int32_t* super_first,
                               double* const* blk_ptr, const int32_t* blk_ld,
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
                blk_ptr[b][lu + size_t(lv) * blk_ld[b]] = vals[t];
                break;
            }
    }
}

void launch_leaf_scatter(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                         const int32_t* iperm, const int32_t* pos_super,
                         const int32_t* super_first, double* const* blk_ptr,
                         const int32_t* blk_ld, const int32_t* blk_col,
                         const int32_t* blk_begin, int n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_leaf_scatter, dim3((n + NT - 1) / NT), dim3(NT), 0, s, row_ptr,
                       col_idx, vals, iperm, pos_super, super_first, blk_ptr, blk_ld, blk_col,
                       blk_begin, n);
    check_launch("k_leaf_scatter");
}

// ---------------------------------------------------------------------------------
// Solve phase: forward (gather form) and backward sweeps of one colour
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_fwd(const FwdTarget* targets, const FwdContrib* contrib,
                                            double* V, int64_t ldv, int nrhs) {
    const FwdTarget t = targets[blockIdx.x];
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    __shared__ double part[NT / WAVE][WAVE];
    for (int c = 0; c < nrhs; ++c) {
        double* Vc = V + size_t(c) * ldv;
        for (int r0 = 0; r0 < t.len; r0 += WAVE) {
            const int i = r0 + lane;
            double acc = 0.0;
            if (i < t.len) {
                for (int q = t.c_begin; q < t.c_end; ++q) {
                    const FwdContrib f = contrib[q];
                    const double* x = Vc + f.src;
                    for (int j = wv; j < f.m; j += NT / WAVE)
                        acc += f.G[i + size_t(j) * f.ldG] * x[j];
                }
            }
            part[wv][lane] = acc;
            __syncthreads();
            if (wv == 0 && i < t.len) {
                double s = 0.0;
                for (int w = 0; w < NT / WAVE; ++w) s += part[w][lane];
                Vc[t.dst + i] += t.sign * s;
            }
            __syncthreads();
        }
    }
}

void launch_fwd(const FwdTarget* t, const FwdContrib* c, int nt, double* V, int64_t ldv,
                int nrhs, double bytes, hipStream_t s) {
    if (nt <= 0) return;
    ProfScope ps("k_fwd", bytes, s);
    hipLaunchKernelGGL(k_fwd, dim3(nt), dim3(NT), 0, s, t, c, V, ldv, nrhs);
    check_launch("k_fwd");
}

constexpr int BWD_MAX_ROWS = 6144;

__global__ __launch_bounds__(NT) void k_bwd(const BwdNode* nodes, const BwdSeg* segs, double* V,
                                            int64_t ldv, int nrhs) {
    const BwdNode nd = nodes[blockIdx.x];
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    __shared__ double v[BWD_MAX_ROWS];
    for (int c = 0; c < nrhs; ++c) {
        double* Vc = V + size_t(c) * ldv;
        int pos = 0;
        for (int q = nd.seg_begin; q < nd.seg_end; ++q) {
            const BwdSeg sg = segs[q];
            for (int i = threadIdx.x; i < sg.len; i += NT) v[pos + i] = sg.sign * Vc[sg.off + i];
            pos += sg.len;
        }
        __syncthreads();
        for (int j = wv; j < nd.m; j += NT / WAVE) {
            const double* g = nd.G + size_t(j) * nd.ldG;
            double acc = 0.0;
            for (int i = lane; i < nd.rows; i += WAVE) acc += g[i] * v[i];
            acc = wave_sum(acc);
            if (lane == 0) Vc[nd.dst + j] = acc;
        }
        __syncthreads();
    }
}

void launch_bwd(const BwdNode* nodes, const BwdSeg* segs, int nn, double* V, int64_t ldv,
                int nrhs, int max_rows, double bytes, hipStream_t s) {
    if (nn <= 0) return;
    ProfScope ps("k_bwd", bytes, s);
    if (max_rows > BWD_MAX_ROWS) throw Error{HSOLVE_ERR_INVALID, "factor block too tall for k_bwd"};
    hipLaunchKernelGGL(k_bwd, dim3(nn), dim3(NT), 0, s, nodes, segs, V, ldv, nrhs);
    check_launch("k_bwd");
}

// ---------------------------------------------------------------------------------
// Permutations, SpMV, BLAS-1
// ---------------------------------------------------------------------------------
__global__ void k_gather_perm(const double* src, int lds, double* dst, int64_t ldd,
                              const int32_t* perm, int n, int nrhs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    for (int c = 0; c < nrhs; ++c) dst[p + c * ldd] = src[u + size_t(c) * lds];
}

void launch_gather_perm(const double* src, int lds, double* dst, int64_t ldd, const int32_t* perm,
                        int n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_perm, dim3((n + NT - 1) / NT), dim3(NT), 0, s, src, lds, dst,
                       ldd, perm, n, nrhs);
    check_launch("k_gather_perm");
}

__global__ void k_scatter_perm(const double* src, int64_t lds, double* dst, int ldd,
                               const int32_t* perm, int n, int nrhs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int u = perm[p];
    for (int c = 0; c < nrhs; ++c) dst[u + size_t(c) * ldd] = src[p + c * lds];
}

void launch_scatter_perm(const double* src, int64_t lds, double* dst, int ldd,
                         const int32_t* perm, int n, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_perm, dim3((n + NT - 1) / NT), dim3(NT), 0, s, src, lds, dst,
                       ldd, perm, n, nrhs);
    check_launch("k_scatter_perm");
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

constexpr int DOT_BLOCKS = 512;

__global__ __launch_bounds__(NT) void k_dot2_part(const double* a, const double* b,
                                                  const double* c, const double* d, int n,
                                                  double* part) {
    __shared__ double red[NT / WAVE];
    double s0 = 0.0, s1 = 0.0;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        s0 += a[i] * b[i];
        if (c) s1 += c[i] * d[i];
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0;
        part[2 * blockIdx.x + 1] = s1;
    }
}

__global__ __launch_bounds__(NT) void k_dot2_final(const double* part, int nb, double* out) {
    __shared__ double red[NT / WAVE];
    double s0 = 0.0, s1 = 0.0;
    for (int i = threadIdx.x; i < nb; i += NT) {
        s0 += part[2 * i];
        s1 += part[2 * i + 1];
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
    }
}

void launch_dot2(const double* a, const double* b, const double* c, const double* d, int n,
                 double* out, hipStream_t s) {
    // out[2 .. 2 + 2*DOT_BLOCKS) is used as partial-sum scratch
    int nb = (n + NT - 1) / NT;
    nb = nb < 1 ? 1 : (nb > DOT_BLOCKS ? DOT_BLOCKS : nb);
    hipLaunchKernelGGL(k_dot2_part, dim3(nb), dim3(NT), 0, s, a, b, c, d, n, out + 2);
    check_launch("k_dot2_part");
    hipLaunchKernelGGL(k_dot2_final, dim3(1), dim3(NT), 0, s, out + 2, nb, out);
    check_launch("k_dot2_final");
}

__global__ void k_axpy2(double* x, const double* p, double* r, const double* q,
                        const double* ratio, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = ratio[0] / ratio[1];
    x[i] += a * p[i];
    r[i] -= a * q[i];
}

void launch_axpy2(double* x, const double* p, double* r, const double* q, const double* alpha,
                  int n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy2, dim3((n + NT - 1) / NT), dim3(NT), 0, s, x, p, r, q, alpha, n);
    check_launch("k_axpy2");
}

__global__ void k_xpby(double* p, const double* z, const double* ratio, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    p[i] = z[i] + (ratio[0] / ratio[1]) * p[i];
}

void launch_xpby(double* p, const double* z, const double* beta, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_xpby, dim3((n + NT - 1) / NT), dim3(NT), 0, s, p, z, beta, n);
    check_launch("k_xpby");
}

__global__ void k_fill(double* p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

void launch_fill(double* p, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = (n + NT - 1) / NT;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_fill, dim3(unsigned(nb)), dim3(NT), 0, s, p, v, n);
    check_launch("k_fill");
}

}  // namespace hs
