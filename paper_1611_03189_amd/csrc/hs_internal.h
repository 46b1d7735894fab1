// Internal data structures of the hsolve library (host side) and the launch wrappers of
// its HIP kernels. Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hsolve.h"

namespace hs {

// ---------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------
struct Error {
    hsolve_status status;
    std::string what;
};

#define HS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::hs::Error{e_ == hipErrorOutOfMemory ? HSOLVE_ERR_OOM               \
                                                        : HSOLVE_ERR_DEVICE,          \
                              std::string(#call) + ": " + hipGetErrorString(e_)};     \
    } while (0)

// ---------------------------------------------------------------------------------
// Device memory: bump allocators over parts of the caller's arena (256-byte aligned).
// In a dry run (base == nullptr) a region only counts bytes: the analysis replays the
// factorization's allocations with upper-bound sizes to size the arena.
// ---------------------------------------------------------------------------------
class Region {
public:
    void init(char* base, size_t cap, const char* name) {
        base_ = base;
        cap_ = cap;
        name_ = name;
        off_ = high_ = 0;
    }
    void* alloc(size_t bytes);
    template <class T> T* alloc_n(size_t n) { return static_cast<T*>(alloc(n * sizeof(T))); }
    void reset() { off_ = 0; }     // reuse from the start (stream order keeps this safe)
    size_t high_water() const { return high_; }
    size_t in_use() const { return off_; }
    size_t capacity() const { return cap_; }
    char* base() const { return base_; }
    char* top() const { return base_ + off_; }

private:
    char* base_ = nullptr;
    size_t cap_ = 0, off_ = 0, high_ = 0;
    const char* name_ = "";
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Pinned host staging + device copy of small task tables.
class Staging {
public:
    ~Staging();
    // copies `bytes` from src into pinned memory and enqueues an H2D copy into dst_pool;
    // returns the device pointer. In a dry run only the device bytes are counted.
    void* upload(const void* src, size_t bytes, Region& dst_pool, hipStream_t s);
    template <class T> T* upload_vec(const std::vector<T>& v, Region& pool, hipStream_t s) {
        if (v.empty()) return nullptr;
        return static_cast<T*>(upload(v.data(), v.size() * sizeof(T), pool, s));
    }
    // Batched uploads: between begin_batch and end_batch the copies of uploads that are
    // contiguous both in pinned memory and on the device merge into one, issued when the run
    // breaks or at end_batch. Nothing may read the tables before end_batch.
    void begin_batch() { batch_ = true; }
    void end_batch(hipStream_t s) {
        flush_pending(s);
        batch_ = false;
    }
    void reset();   // only after a stream synchronisation; drops a batch an error left open

private:
    void flush_pending(hipStream_t s);
    char* host_ = nullptr;
    size_t cap_ = 0, off_ = 0;
    bool batch_ = false;
    char* pend_h_ = nullptr;
    char* pend_d_ = nullptr;
    size_t pend_bytes_ = 0;

public:
    bool dry = false;
};

// ---------------------------------------------------------------------------------
// Optional per-kernel timing: HIP events recorded on the launch stream around every
// launch while a profile is active on the calling thread
// ---------------------------------------------------------------------------------
struct ProfRec {
    const char* name;
    double work;             // algorithmic flops (compute kernels) or bytes (memory kernels)
    hipEvent_t a, b;
};

struct ProfTotal {
    std::string name;
    double ms = 0.0, work = 0.0;
    int64_t launches = 0;
};

class Profiler {
public:
    ~Profiler();
    bool on = false;
    std::string only;                  // record only launches of this kernel name (empty: all)
    void clear();
    void record(const char* name, double work, hipEvent_t a, hipEvent_t b);
    hipEvent_t event();
    std::vector<ProfTotal> totals();   // synchronises; aggregates by kernel name

private:
    std::vector<ProfRec> recs_;
    std::vector<hipEvent_t> pool_;
    size_t used_ = 0;
};

extern thread_local Profiler* t_prof;

struct ProfScope {           // brackets one launch
    ProfScope(const char* name, double work, hipStream_t s);
    ~ProfScope();
    const char* name;
    double work;
    hipStream_t s;
    hipEvent_t a = nullptr;
};

// ---------------------------------------------------------------------------------
// Symbolic schedule of one level (depth d): super nodes are the 2^d clusters of depth d
// ---------------------------------------------------------------------------------
struct LevelSym {
    int d = 0;
    std::vector<std::vector<int>> colours;
    std::vector<int> colour_of;                 // -1 for empty super nodes
    std::vector<std::vector<int>> N, W;         // neighbour / well-separated partners
    std::vector<std::vector<uint8_t>> Nred, Wred;  // partner already red at elimination
    std::vector<uint8_t> super_nonempty, red_nonempty;
    std::vector<std::vector<int>> init_partners;   // block pattern when the level starts
};

// ---------------------------------------------------------------------------------
// Dense blocks of the current matrix (column-major, canonical orientation i <= j)
// ---------------------------------------------------------------------------------
struct Block {               // elements of the factorization's storage type (double or float)
    void* p = nullptr;
    int rows = 0, cols = 0, ld = 0;
};

inline uint64_t bkey(int i, int j) {
    return (uint64_t(uint32_t(i)) << 32) | uint32_t(j);
}

// ---------------------------------------------------------------------------------
// Numeric factor of one eliminated super node, kept for the solve phase:
// Gm = [M_ss (m rows); T_N = A_Ns M_ss (ntot rows); P_ss (k rows)], m columns,
// column-major with ld = m + ntot + k.
// ---------------------------------------------------------------------------------
struct NodeNum {
    int m = 0, k = 0, ntot = 0, ka = 0;
    void* Gm = nullptr;        // in the factorization's storage type
    float* Gm32 = nullptr;     // what the FP32 solve phase reads: a rounded copy of an FP64 factor,
                               // or the FP32 factor itself
    int ldG = 0;
    std::vector<int> noff;     // row offset of each neighbour inside T_N
};

struct LevelNum {
    std::vector<int> msz, ksz;          // super / red sizes (2^d)
    std::vector<int64_t> red_off;       // start of each red segment in the solve vector
    std::vector<NodeNum> node;
};

// ---------------------------------------------------------------------------------
// Kernel task records (shared layout with kernels.hip)
// ---------------------------------------------------------------------------------
struct CopyTask {            // dst(i,j) = src(i,j) or src(j,i) (trans), in the launch's type
    const void* src;
    void* dst;
    int lds, ldd, rows, cols, trans, pad;
};

// Flags of a GEMM task (for C) and term (for B): GEMM_REL, the pointer field holds an element
// offset from one of the two base pointers the launch passes (GEMM_BASE1 picks the second);
// GEMM_NEG (term), the term enters with a minus sign. GEMM_MIRROR (task, square and
// symmetric C such as A A^T): the tiles wholly above the diagonal (tj TN >= ti TM + TM) are not
// listed, and every element (i, j) whose transposed position lies in one of them is also
// written to (j, i).
enum { GEMM_NEG = 1, GEMM_REL = 2, GEMM_BASE1 = 4, GEMM_MIRROR = 8 };

struct GemmTask {            // C = beta C + alpha sum_t op(A_t) op(B_t), C is M x N (launch's type)
    void* C;
    int ldc, M, N, t_begin, t_end, flags;
    double alpha, beta;
};

struct GemmTerm {
    const void* A;
    const void* B;
    int lda, ldb, K, transA, transB, flags;
};

struct GemmTile {            // one output tile of a task (the launch's tile shape)
    int task, ti, tj, pad;
};

// Tile shapes of the grouped GEMM and the autotuned choice per size bucket. A launch's bucket
// is decided by its number of 64 x 64 output tiles and its mean inner dimension.
struct GemmShape {
    int tm, tn, tk;
    int persistent;          // 1: a grid of resident workgroups loops over the tiles
};
constexpr int GEMM_VARIANTS = 8;
extern const GemmShape GEMM_SHAPES[GEMM_VARIANTS];
constexpr int GEMM_TILE_BUCKETS = 4;       // 64x64 tiles: < 32, < 256, < 2048, more
constexpr int GEMM_K_BUCKETS = 3;          // mean K: <= 64, <= 256, more
constexpr int GEMM_BUCKETS = GEMM_TILE_BUCKETS * GEMM_K_BUCKETS;
int gemm_bucket(double tiles64, double mean_k);
int gemm_variant(int bucket, bool f32);    // the tuned choice (0 until tuned)
void set_gemm_variant(int bucket, bool f32, int variant);
size_t tune_workspace_bytes();
void tune_gemm(void* d_work, size_t bytes, hipStream_t st, int* choice, double* ms);

struct CholTask {            // in: A (m x m, SPD); out: Ainv (m x m) = A^{-1} (launch's type)
    void* A;
    void* Ainv;
    void* work;              // m x m scratch for blocks too large for LDS (else null)
    long long* tstamp;       // optional: 4 clock stamps at phase boundaries and 5 per-phase cycle sums of the panels (trace only)
    int lda, ldi, m, id;
};

struct CompressTask {
    const double* G;         // m x m Gram matrix A_sw A_sw^T (ld m), consumed
    const double* Z;         // m x nz vectors to keep [phi_s, A_sw phi_w] (ld m), or null
    double* work;            // scratch: m^2 + 32 m + 64 doubles
    double* U;               // out: m x k (ld m)
    long long* tstamp;       // optional: 8 clock stamps at phase boundaries (trace only)
    int m, nz, wt, id;
};

struct FwdTarget {           // V[dst + i] += sign * sum_c Gc[i, :] V[src_c + :]
    long long dst;
    int len, sign, c_begin, c_end;
};

struct FwdContrib {
    const void* G;           // first row of the contributing rows, column-major (double or float)
    long long src;           // start of phi_s in V
    int ldG, m;
};

struct BwdNode {             // x_s = Gm^T [phi_s; -x_N; x_r], written at dst of X
    const void* G;           // double or float, as the solve vectors
    long long dst;
    int ldG, m, rows, seg_begin, seg_end, pad;
};

struct DemoteTask {          // dst[i] = float(src[i]), i < count
    const double* src;
    float* dst;
    long long count;
};

struct PromoteTask {         // dst[i] = double(src[i]), i < count
    const float* src;
    double* dst;
    long long count;
};

struct BwdSeg {              // sign * (buf ? X : V)[off .. off + len)
    long long off;
    int len, sign, buf, pad;
};

// ---------------------------------------------------------------------------------
// The plan
// ---------------------------------------------------------------------------------
struct Plan {
    // pattern and options
    int n = 0;
    int64_t nnz = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col_idx;
    hsolve_options opt{};
    std::vector<double> coords, phi;   // copies (phi column-major n x nvec)
    int nphi = 0;                      // preserved vectors (0 for LoRaSp)
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;        // factorization: pivot blocks beside the compression
    hipEvent_t ev_ready = nullptr, ev_done = nullptr;
    hipStream_t side2 = nullptr;       // factorization: large nodes' compression beside the small ones'
    hipEvent_t ev_ready2 = nullptr, ev_done2 = nullptr;

    // tree
    int L = 0;
    std::vector<int32_t> perm, iperm, leaf_off;   // leaf order
    std::vector<LevelSym> sym;                     // sym[d], d = 0 .. L-1
    int total_colours = 0;

    // pattern in pinned host memory (copied into the arena by every factorization)
    int64_t* h_row_ptr = nullptr;
    int32_t* h_col_idx = nullptr;
    int32_t* h_perm = nullptr;         // [perm (n) | iperm (n) | super node of each position (n)]
    // device copies of the pattern, in the arena
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col_idx = nullptr;
    double* d_values = nullptr;
    int32_t* d_perm = nullptr;         // [perm (n) | iperm (n)]
    int32_t* d_iperm = nullptr;        // = d_perm + n
    int32_t* d_pos_super = nullptr;    // super node of the first level for each position

    // numeric factor
    bool factored = false;
    bool dry = false;                  // replaying the factorization to size the arena
    std::vector<LevelNum> num;         // num[d]
    int64_t vlen = 0;                  // length of one solve-vector column
    // Arena layout: [pattern | factor data + apply schedule (fpool, grows up) ... |
    //                live blocks of even depths | of odd depths | per-colour scratch]
    // The three transient regions have the capacities the dry run of the analysis found;
    // after the factorization they are free, and the solve phase takes its vectors from
    // everything above the factor data (wpool).
    char* arena = nullptr;
    size_t arena_bytes = 0;
    size_t pattern_bytes = 0;          // device bytes of the pattern part
    size_t cap_live[2] = {0, 0}, cap_scratch = 0;   // transient capacities (dry run)
    size_t bound_factor = 0;           // dry-run high water of the factor region
    size_t arena_bound = 0;            // what hsolve_analyze reports
    int* h_flags = nullptr;            // pinned: pivot failure flags + ranks of a colour
    Region fpool;                      // factor data and apply schedule (kept)
    Region lpool[2];                   // live blocks by depth parity
    Region spool;                      // per-colour scratch
    Region wpool;                      // solve phase: vectors and Krylov workspace
    Staging stage;

    // apply schedule (device), per level and colour
    struct ApplyGemm {      // one sweep of a colour as grouped-GEMM tables (vector-relative)
        GemmTask* tasks = nullptr;
        GemmTerm* terms = nullptr;
        GemmTile* tiles = nullptr;
        int ntiles = 0;
        double flops = 0.0;  // per right-hand side
    };
    struct ColourSched {
        double fwd_bytes = 0.0, bwd_bytes = 0.0;   // algorithmic bytes per rhs
        FwdTarget* fwd_t = nullptr; int nfwd = 0; int max_len = 0;
        FwdContrib* fwd_c = nullptr;
        BwdNode* bwd_n = nullptr; int nbwd = 0; int max_m = 0;
        BwdSeg* bwd_s = nullptr;
        ApplyGemm gf, gb;   // the same sweeps for several right-hand sides
    };
    std::vector<std::vector<ColourSched>> sched;   // sched[d][c]
    bool apply32 = false;                           // solve phase in single precision
    bool f32 = false;                               // factorization in single precision
    void* d_V = nullptr;                            // forward right-hand sides (phi)
    void* d_X = nullptr;                            // backward solutions (x)
    int V_cols = 0;
    double* h_scalars = nullptr;                    // pinned
    double* d_krylov = nullptr;                     // PCG vectors (R, Z, P, Q, X blocks)
    double* d_kscal = nullptr;                      // PCG scalars per column + dot partials
    int* d_kflag = nullptr;                         // PCG: column still iterating
    int krylov_cols = 0;
    double* d_gmres = nullptr;                      // GMRES: V (restart+1), Z (restart), w, r, x
    int gmres_restart = 0;
    int h_scalar_cols = 0;
    struct Graph {                                  // captured apply sweeps for one workspace
        const void* V;
        const void* X;
        int nrhs;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t cap = nullptr;                      // capture stream of the sweeps

    // arena bytes used by the last factorization and its solves
    size_t device_bytes() const {
        if (!arena) return 0;
        return pattern_bytes + fpool.high_water() +
               std::max(cap_live[0] + cap_live[1] + cap_scratch, wpool.high_water());
    }
    hsolve_stats stats{};
    Profiler prof;
    std::vector<ProfTotal> prof_totals;
    ~Plan();
};

// analyze.hip (host only)
void analyze(Plan& P);
// runtime.hip
void pin_pattern(Plan& P);                       // pinned host copy of the pattern (analysis)
void bind_arena(Plan& P, void* arena, size_t bytes);   // carve the regions, upload the pattern
size_t solve_ws_bytes(const Plan& P, int nrhs, int krylov);   // solve-phase workspace
int solve_batch(const Plan& P, int nrhs, int krylov);          // columns per batch that fit
// factor.hip: the numeric factorization; with P.dry set, a replay on the host that only
// counts the bytes of every allocation, with upper-bound sizes (no GPU work)
void factor(Plan& P, const double* values);
void size_arena(Plan& P);
double level_eps(const Plan& P, int d);          // compression tolerance of depth d
// solve.hip
void build_apply_schedule(Plan& P);
void begin_workspace(Plan& P);
constexpr size_t APPLY_SCRATCH_BYTES = size_t(64) << 20;   // static scratch of hsolve_apply_static
void apply_static(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz);
void apply(Plan& P, int nrhs, const double* r, int ldr, double* z, int ldz, bool graph = true);
void clear_graphs(Plan& P);      // drop the captured sweeps (factor, destroy)
void pcg(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
         bool flexible, int* its, double* rel);
void stationary(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
                int* its, double* rel);
void gmres(Plan& P, int nrhs, const double* b, int ldb, double* x, int ldx, double tol, int max_iter,
           int restart, int* its, double* rel);
void spmv(Plan& P, const double* x, double* y);

// kernels.hip: launch wrappers (all asynchronous on stream s)
// the factorization's kernels in its storage type T (double, or float with factor_prec = 32)
template <typename T>
void launch_copy(const CopyTask* d_tasks, int ntasks, int max_cols, double bytes, hipStream_t s);
template <typename T>
// base0, base1: the bases of GEMM_REL pointers; ncols > 0 overrides every task's N (the
// launch then covers columns [0, ncols) of relative operands); name: the profiler's label
void launch_gemm(const GemmTask* d_tasks, const GemmTerm* d_terms, const GemmTile* d_tiles,
                 int ntiles, double flops, int variant, hipStream_t s, T* base0 = nullptr,
                 T* base1 = nullptr, int ncols = 0, const char* name = nullptr);
template <typename T>
void launch_chol_inv(const CholTask* d_tasks, int ntasks, int* d_fail, double flops, bool lds,
                     int max_m, hipStream_t s);
void launch_promote(const PromoteTask* d_tasks, int ntasks, double elems, hipStream_t s);
// d_rank[id] = |U1| + k2 (the kept count); with kx_max > 0 also d_extra[id] = kx, the
// eigenvectors past the threshold written after the kept ones (U columns rank .. rank + kx)
void launch_compress(const CompressTask* d_tasks, int ntasks, int variant, double eps,
                     int* d_rank, int* d_extra, int kx_max, double flops, bool lds, int max_m,
                     int force_lpe, int force_vectors, hipStream_t s);
// Rayleigh-Ritz on a window W (m x s, ld ldw, s <= RITZ_MAX) of the basis, given B = W^T A_sw
// (s x wt, ld s): W's first w columns become the eigenvectors of B B^T of the w largest
// eigenvalues, mapped by W
constexpr int RITZ_MAX = 16;
constexpr int RITZ_KEEP = 8, RITZ_EXTRA = 8;   // window: kept directions, and those past the threshold
struct RitzTask {
    const double* B;
    double* W;
    int s, w, wt, m, ldw;
};
void launch_comp_ritz(const RitzTask* d_tasks, int ntasks, hipStream_t s);
// Appendix B first-order one-sided projection: Z (m x nz <= 16) becomes its left singular
// vectors above eps1 sigma_1(Z), zero columns after them
void launch_gc_truncate(const CompressTask* d_tasks, int ntasks, double eps1, hipStream_t s);
constexpr int LDS_MAX_M = 128;   // compression blocks up to this size work in LDS
constexpr int CMP_WY_NB = 16;     // reflectors per block in the compression back-transformation
// doubles of the per-node compression work buffer for a super node of m unknowns
inline size_t cmp_work_doubles(int m) {
    return size_t(m) * m + 32 * size_t(m) + 64 + size_t(CMP_WY_NB) * CMP_WY_NB * ((m + CMP_WY_NB - 1) / CMP_WY_NB) +
           4 * size_t(m) * (size_t(m + 63) / 64 * 64);
}
constexpr int PIV_LDS_MAX_M = 64; // pivot blocks up to this size are factored in LDS; larger
                                  // ones by the blocked kernel (panels of 32 columns)
template <typename T>
void launch_leaf_scatter(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                         const int32_t* iperm, const int32_t* pos_super,
                         const int32_t* super_first, void* const* blk_ptr,
                         const int32_t* blk_ld, const int32_t* blk_col,
                         const int32_t* blk_begin, int n, hipStream_t s);
// solve phase in the storage type T of the factor copy it reads (double, or float for the
// single-precision solve); vectors enter and leave it in double
template <typename T>
void launch_fwd(const FwdTarget* t, const FwdContrib* c, int nt, int max_len, T* V,
                int64_t ldv, int nrhs, double bytes, hipStream_t s);
template <typename T>
void launch_bwd(const BwdNode* nodes, const BwdSeg* segs, int nn, int max_m, const T* V,
                T* X, int64_t ldv, int nrhs, double bytes, hipStream_t s);
template <typename T>
void launch_gather_perm(const double* src, int lds, T* dst, int64_t ldd, const int32_t* perm,
                        int n, int nrhs, hipStream_t s);   // dst[p] = src[perm[p]]
template <typename T>
void launch_scatter_perm(const T* src, int64_t lds, double* dst, int ldd,
                         const int32_t* perm, int n, int nrhs, hipStream_t s); // dst[perm[p]] = src[p]
void launch_demote(const DemoteTask* d_tasks, int ntasks, double elems, hipStream_t s);
void launch_spmv(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                 const double* x, double* y, int n, int64_t nnz, hipStream_t s);
constexpr int DOTM_BLOCKS = 512;   // partial sums per column of a batched dot product
constexpr int MAX_SUPER = 512;     // largest super node the compression and pivot kernels take
void launch_spmv_multi(const int64_t* row_ptr, const int32_t* col_idx, const double* vals,
                       const double* X, int64_t ldx, double* Y, int64_t ldy, int n, int nrhs,
                       int64_t nnz, hipStream_t s);
void launch_dots(const double* A, const double* B, int64_t ld, int n, int nrhs, double* part, double* out,
                 hipStream_t s);    // out[c] = A(:, c) . B(:, c); part: DOTM_BLOCKS * nrhs scratch
void launch_axpy2_multi(double* X, const double* P, double* R, const double* Q, int64_t ld, int n, int nrhs,
                        const double* num, const double* den, const int* active, hipStream_t s);
void launch_xpby_multi(double* P, const double* Z, int64_t ld, int n, int nrhs, const double* num,
                       const double* sub, const double* den, const int* active, hipStream_t s);
void launch_pcg_flags(const double* rr, const double* nb, double tol, int* active, double* dst,
                      const double* src, int nrhs, hipStream_t s);
void launch_copy_scalars(double* dst, const double* src, int n, hipStream_t s);
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s);
void launch_check_finite(const double* v, int64_t n, int* flag, hipStream_t s);   // *flag = any non-finite
// restarted GMRES: y += sign * (*a) * x; y = s * x; r = b - w; x += Z y (y: device, k entries)
void launch_axpy_dev(double* y, const double* x, const double* a, double sign, int n, hipStream_t s);
// stationary iteration, active columns only: X += Z; R = B - Q
void launch_add_multi(double* X, const double* Z, int64_t ld, int n, int nrhs, const int* active, hipStream_t s);
void launch_sub_multi(double* R, const double* B, int64_t ldb, const double* Q, int64_t ld, int n, int nrhs,
                      const int* active, hipStream_t s);
void launch_scale(double* y, const double* x, double sc, int n, hipStream_t s);
void launch_sub(double* r, const double* b, const double* w, int n, hipStream_t s);
void launch_gemv_acc(double* x, const double* Z, int64_t ldz, const double* y, int k, int n, hipStream_t s);

}  // namespace hs
