// Autotuner of the grouped GEMM's tile shape. A launch is classified by its number of
// 64 x 64 output tiles (its size in workgroups of the default shape) and by its mean
// inner dimension (how long each tile accumulates). For each such bucket the tuner times
// every tile shape on a synthetic launch of that size (groups of 128 x 128 products with the
// bucket's inner dimension, operands spread over the caller's workspace) and keeps the
// fastest. The choice holds for the whole process; all shapes give the same bits.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <vector>

#include "hs_internal.h"

namespace hs {

namespace {
std::atomic<int> g_variant[2][GEMM_BUCKETS];   // [FP64, FP32]; zero-initialised: 64 x 64 x 16

constexpr int TILE_REP[GEMM_TILE_BUCKETS] = {16, 128, 1024, 4096};   // 64 x 64 tiles per launch
constexpr int K_REP[GEMM_K_BUCKETS] = {32, 160, 512};
constexpr int TASK_M = 128;                 // synthetic products are 128 x 128 x K
}  // namespace

int gemm_bucket(double tiles64, double mean_k) {
    const int tb = tiles64 < 32 ? 0 : tiles64 < 256 ? 1 : tiles64 < 2048 ? 2 : 3;
    const int kb = mean_k <= 64 ? 0 : mean_k <= 256 ? 1 : 2;
    return tb * GEMM_K_BUCKETS + kb;
}

int gemm_variant(int bucket, bool f32) {
    if (bucket < 0 || bucket >= GEMM_BUCKETS) return 0;
    return g_variant[f32][bucket].load(std::memory_order_relaxed);
}

void set_gemm_variant(int bucket, bool f32, int variant) {
    if (bucket >= 0 && bucket < GEMM_BUCKETS && variant >= 0 && variant < GEMM_VARIANTS)
        g_variant[f32][bucket].store(variant, std::memory_order_relaxed);
}

size_t tune_workspace_bytes() {
    // C: the largest launch's 128 x 128 outputs; A, B: 32 distinct 128 x 512 operands each
    const size_t tasks = size_t(TILE_REP[GEMM_TILE_BUCKETS - 1]) / 4;
    return sizeof(double) * (tasks * TASK_M * TASK_M + 2 * 32 * size_t(TASK_M) * K_REP[GEMM_K_BUCKETS - 1]) +
           (size_t(4) << 20);
}

// Times every shape on every bucket, in FP64 and then in FP32 (the FP32 factorization's
// GEMMs); ms[(t * GEMM_BUCKETS + b) * GEMM_VARIANTS + v] receives the best of three launches,
// choice[t * GEMM_BUCKETS + b] the fastest shape (also stored for the process), t = 0 FP64,
// 1 FP32.
template <typename T>
static void tune_type(char* w, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int* choice, double* ms);

void tune_gemm(void* d_work, size_t bytes, hipStream_t st, int* choice, double* ms) {
    if (bytes < tune_workspace_bytes())
        throw Error{HSOLVE_ERR_OOM, "tuning workspace too small: needs " + std::to_string(tune_workspace_bytes())};
    char* w = static_cast<char*>(d_work);
    hipEvent_t e0, e1;
    HS_HIP(hipEventCreate(&e0));
    HS_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    tune_type<double>(w, st, e0, e1, choice, ms);
    tune_type<float>(w, st, e0, e1, choice ? choice + GEMM_BUCKETS : nullptr,
                     ms ? ms + GEMM_BUCKETS * GEMM_VARIANTS : nullptr);
    HS_HIP(hipStreamSynchronize(st));
}


template <typename T>
static void tune_type(char* w, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int* choice, double* ms) {
    constexpr bool F32 = sizeof(T) == 4;
    const int kmax = K_REP[GEMM_K_BUCKETS - 1];
    T* A = reinterpret_cast<T*>(w);
    T* B = A + 32 * size_t(TASK_M) * kmax;
    T* C = B + 32 * size_t(TASK_M) * kmax;
    char* tables = reinterpret_cast<char*>(C + size_t(TILE_REP[GEMM_TILE_BUCKETS - 1]) / 4 * TASK_M * TASK_M);
    launch_fill<T>(A, T(0.5), 64 * int64_t(TASK_M) * kmax, st);
    launch_fill<T>(C, T(0), int64_t(TILE_REP[GEMM_TILE_BUCKETS - 1]) / 4 * TASK_M * TASK_M, st);
    for (int tb = 0; tb < GEMM_TILE_BUCKETS; ++tb)
        for (int kb = 0; kb < GEMM_K_BUCKETS; ++kb) {
            const int bucket = tb * GEMM_K_BUCKETS + kb;
            const int ntask = std::max(1, TILE_REP[tb] / 4), K = K_REP[kb];
            std::vector<GemmTask> tk(ntask);
            std::vector<GemmTerm> tm(ntask);
            for (int t = 0; t < ntask; ++t) {
                tk[t] = GemmTask{C + size_t(t) * TASK_M * TASK_M, TASK_M, TASK_M, TASK_M, t, t + 1, 0, -1.0, 1.0};
                tm[t] = GemmTerm{A + size_t(t % 32) * TASK_M * kmax, B + size_t((t * 7) % 32) * TASK_M * kmax,
                                 TASK_M, TASK_M, K, 0, 1, 0};
            }
            double best = 1e300;
            int arg = 0;
            for (int v = 0; v < GEMM_VARIANTS; ++v) {
                const GemmShape sh = GEMM_SHAPES[v];
                std::vector<GemmTile> tl;
                for (int t = 0; t < ntask; ++t)
                    for (int i = 0; i * sh.tm < TASK_M; ++i)
                        for (int j = 0; j * sh.tn < TASK_M; ++j) tl.push_back(GemmTile{t, i, j, 0});
                const size_t o1 = align256(sizeof(GemmTask) * tk.size());
                const size_t o2 = o1 + align256(sizeof(GemmTerm) * tm.size());
                HS_HIP(hipMemcpyAsync(tables, tk.data(), sizeof(GemmTask) * tk.size(), hipMemcpyHostToDevice, st));
                HS_HIP(hipMemcpyAsync(tables + o1, tm.data(), sizeof(GemmTerm) * tm.size(), hipMemcpyHostToDevice, st));
                HS_HIP(hipMemcpyAsync(tables + o2, tl.data(), sizeof(GemmTile) * tl.size(), hipMemcpyHostToDevice, st));
                const auto* dt = reinterpret_cast<const GemmTask*>(tables);
                const auto* dm = reinterpret_cast<const GemmTerm*>(tables + o1);
                const auto* dl = reinterpret_cast<const GemmTile*>(tables + o2);
                launch_gemm<T>(dt, dm, dl, int(tl.size()), 0.0, v, st);      // warm-up
                float t_best = 1e30f;
                for (int rep = 0; rep < 3; ++rep) {
                    HS_HIP(hipEventRecord(e0, st));
                    launch_gemm<T>(dt, dm, dl, int(tl.size()), 0.0, v, st);
                    HS_HIP(hipEventRecord(e1, st));
                    HS_HIP(hipEventSynchronize(e1));
                    float t = 0.f;
                    HS_HIP(hipEventElapsedTime(&t, e0, e1));
                    t_best = std::min(t_best, t);
                }
                if (ms) ms[bucket * GEMM_VARIANTS + v] = t_best;
                if (t_best < best) {
                    best = t_best;
                    arg = v;
                }
            }
            set_gemm_variant(bucket, F32, arg);
            if (choice) choice[bucket] = arg;
        }
}

}  // namespace hs
