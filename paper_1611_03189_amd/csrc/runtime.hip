// Device memory pools, pinned staging of task tables, plan teardown.
#include <algorithm>

#include "hs_internal.h"

namespace hs {

void* Region::alloc(size_t bytes) {
    bytes = align256(bytes ? bytes : 1);
    if (off_ + bytes > cap_)
        throw Error{HSOLVE_ERR_OOM, std::string("arena too small: region '") + name_ + "' needs " +
                                        std::to_string(off_ + bytes) + " of " + std::to_string(cap_) +
                                        " bytes (hsolve_analyze reports the bound)"};
    void* p = base_ + off_;
    off_ += bytes;
    if (off_ > high_) high_ = off_;
    return p;
}

Staging::~Staging() {
    if (host_) (void)hipHostFree(host_);
}

void Staging::flush_pending(hipStream_t s) {
    if (!pend_bytes_) return;
    HS_HIP(hipMemcpyAsync(pend_d_, pend_h_, pend_bytes_, hipMemcpyHostToDevice, s));
    pend_bytes_ = 0;
}

// A batch still open here was left by an error: its tables are discarded with it.
void Staging::reset() {
    pend_bytes_ = 0;
    batch_ = false;
    off_ = 0;
}

void* Staging::upload(const void* src, size_t bytes, Region& dst_pool, hipStream_t s) {
    if (dry) return dst_pool.alloc(bytes);
    size_t need = align256(bytes);
    if (off_ + need > cap_) {
        // Growing would move memory that queued copies may still read: callers reset the
        // staging only after a synchronisation, so a fresh, larger buffer is safe to use
        // once the stream has drained (a batch's pending copy is issued first).
        flush_pending(s);
        HS_HIP(hipStreamSynchronize(s));
        size_t ncap = cap_ ? cap_ : (size_t(8) << 20);
        while (ncap < off_ + need || ncap < need) ncap *= 2;
        if (host_) HS_HIP(hipHostFree(host_));
        host_ = nullptr;
        HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_), ncap, hipHostMallocDefault));
        cap_ = ncap;
        off_ = 0;
    }
    char* h = host_ + off_;
    std::memcpy(h, src, bytes);
    off_ += need;
    char* d = static_cast<char*>(dst_pool.alloc(bytes));    // align256(bytes) = need bytes
    if (!batch_) {
        HS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
        return d;
    }
    if (pend_bytes_ && pend_h_ + pend_bytes_ == h && pend_d_ + pend_bytes_ == d) {
        pend_bytes_ += need;
    } else {
        flush_pending(s);
        pend_h_ = h;
        pend_d_ = d;
        pend_bytes_ = need;
    }
    return d;
}

// Pinned host copies of the pattern and leaf order (analysis): every factorization copies
// them into its arena with asynchronous transfers.
void pin_pattern(Plan& P) {
    if (P.h_row_ptr) return;
    const int n = P.n;
    HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_row_ptr), sizeof(int64_t) * (size_t(n) + 1),
                         hipHostMallocDefault));
    HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_col_idx), sizeof(int32_t) * std::max<size_t>(1, P.nnz),
                         hipHostMallocDefault));
    HS_HIP(hipHostMalloc(reinterpret_cast<void**>(&P.h_perm), sizeof(int32_t) * 3 * size_t(n),
                         hipHostMallocDefault));
    std::memcpy(P.h_row_ptr, P.row_ptr.data(), sizeof(int64_t) * (size_t(n) + 1));
    if (P.nnz) std::memcpy(P.h_col_idx, P.col_idx.data(), sizeof(int32_t) * size_t(P.nnz));
    std::memcpy(P.h_perm, P.perm.data(), sizeof(int32_t) * n);
    std::memcpy(P.h_perm + n, P.iperm.data(), sizeof(int32_t) * n);
    int32_t* pos_super = P.h_perm + 2 * size_t(n);
    std::fill(pos_super, pos_super + n, 0);
    if (P.L > 0)
        for (int i = 0; i < (1 << P.L); ++i)
            for (int q = P.leaf_off[i]; q < P.leaf_off[i + 1]; ++q) pos_super[q] = i >> 1;
}

// Carve the caller's arena (see Plan) and enqueue the pattern uploads on the plan's stream.
void bind_arena(Plan& P, void* arena, size_t bytes) {
    char* a = static_cast<char*>(arena);
    const size_t trans = P.cap_live[0] + P.cap_live[1] + P.cap_scratch;
    if (reinterpret_cast<uintptr_t>(a) % 256 != 0)
        throw Error{HSOLVE_ERR_INVALID, "arena not 256-byte aligned"};
    if (bytes < P.pattern_bytes + trans)
        throw Error{HSOLVE_ERR_OOM, "arena too small: " + std::to_string(bytes) + " bytes, the pattern and the "
                                    "transient regions need " + std::to_string(P.pattern_bytes + trans) +
                                    " (bound " + std::to_string(P.arena_bound) + ")"};
    P.arena = nullptr;
    pin_pattern(P);
    P.arena = a;
    P.arena_bytes = bytes;
    const int n = P.n;
    char* q = a;
    P.d_row_ptr = reinterpret_cast<int64_t*>(q);
    q += align256(sizeof(int64_t) * (size_t(n) + 1));
    P.d_col_idx = reinterpret_cast<int32_t*>(q);
    q += align256(sizeof(int32_t) * std::max<size_t>(1, P.nnz));
    P.d_values = reinterpret_cast<double*>(q);
    q += align256(sizeof(double) * std::max<size_t>(1, P.nnz));
    P.d_perm = reinterpret_cast<int32_t*>(q);
    P.d_iperm = P.d_perm + n;
    P.d_pos_super = P.d_perm + 2 * size_t(n);
    char* end = a + bytes;
    char* tbase = end - trans;
    P.fpool.init(a + P.pattern_bytes, size_t(tbase - (a + P.pattern_bytes)), "factor data");
    P.lpool[0].init(tbase, P.cap_live[0], "live blocks (even depths)");
    P.lpool[1].init(tbase + P.cap_live[0], P.cap_live[1], "live blocks (odd depths)");
    P.spool.init(tbase + P.cap_live[0] + P.cap_live[1], P.cap_scratch, "per-colour scratch");
    P.wpool.init(nullptr, 0, "solve workspace");
    hipStream_t st = P.stream;
    HS_HIP(hipMemcpyAsync(P.d_row_ptr, P.h_row_ptr, sizeof(int64_t) * (size_t(n) + 1), hipMemcpyHostToDevice, st));
    if (P.nnz)
        HS_HIP(hipMemcpyAsync(P.d_col_idx, P.h_col_idx, sizeof(int32_t) * size_t(P.nnz), hipMemcpyHostToDevice, st));
    HS_HIP(hipMemcpyAsync(P.d_perm, P.h_perm, sizeof(int32_t) * 3 * size_t(n), hipMemcpyHostToDevice, st));
}

// Device bytes of the solve phase for nrhs columns: the two solve vectors of the sweeps
// (V, X in the storage type of the factor copy) and the outer loop's vectors and scalars
// (krylov < 0: an apply alone). GMRES solves one column at a time.
size_t solve_ws_bytes(const Plan& P, int nrhs, int krylov) {
    const size_t n = size_t(P.n);
    const size_t w = P.apply32 ? sizeof(float) : sizeof(double);
    if (krylov == HSOLVE_GMRES) nrhs = 1;
    size_t b = 2 * align256(w * size_t(P.vlen) * nrhs);
    if (krylov == HSOLVE_GMRES) {
        const size_t m = size_t(std::max(1, P.opt.restart));
        b += align256(sizeof(double) * (n * (2 * m + 4) + (m + 2) + DOTM_BLOCKS + 8));
    } else if (krylov >= 0) {
        b += align256(sizeof(double) * n * 5 * nrhs) + align256(sizeof(double) * size_t(nrhs) * (6 + DOTM_BLOCKS)) +
             align256(sizeof(int) * size_t(nrhs));
    }
    return b;
}

// Right-hand sides per batch: every column of PCG / FPCG / the stationary loop is
// independent, so a call with more columns than the workspace holds runs in batches
// (GMRES runs one column at a time anyway).
int solve_batch(const Plan& P, int nrhs, int krylov) {
    const size_t avail = size_t(P.arena + P.arena_bytes - P.fpool.top());
    if (solve_ws_bytes(P, 1, krylov) > avail)
        throw Error{HSOLVE_ERR_OOM, "arena too small for the solve phase of one right-hand side: needs " +
                                        std::to_string(solve_ws_bytes(P, 1, krylov)) + " bytes above the factor, has " +
                                        std::to_string(avail)};
    if (krylov == HSOLVE_GMRES) return nrhs;
    int lo = 1, hi = nrhs;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (solve_ws_bytes(P, mid, krylov) <= avail) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

thread_local Profiler* t_prof = nullptr;

Profiler::~Profiler() {
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

void Profiler::clear() {
    recs_.clear();
    used_ = 0;
}

hipEvent_t Profiler::event() {
    if (used_ == pool_.size()) {
        hipEvent_t e;
        HS_HIP(hipEventCreate(&e));
        pool_.push_back(e);
    }
    return pool_[used_++];
}

void Profiler::record(const char* name, double work, hipEvent_t a, hipEvent_t b) {
    recs_.push_back(ProfRec{name, work, a, b});
}

std::vector<ProfTotal> Profiler::totals() {
    HS_HIP(hipDeviceSynchronize());
    std::vector<ProfTotal> out;
    for (const ProfRec& r : recs_) {
        float ms = 0.f;
        HS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        ProfTotal* t = nullptr;
        for (auto& x : out)
            if (x.name == r.name) t = &x;
        if (!t) {
            out.push_back(ProfTotal{r.name});
            t = &out.back();
        }
        t->ms += ms;
        t->work += r.work;
        t->launches += 1;
    }
    return out;
}

ProfScope::ProfScope(const char* n, double w, hipStream_t st) : name(n), work(w), s(st) {
    if (t_prof && t_prof->on && (t_prof->only.empty() || t_prof->only == n)) {
        a = t_prof->event();
        HS_HIP(hipEventRecord(a, s));
    }
}

ProfScope::~ProfScope() {
    if (!a) return;
    hipEvent_t b = t_prof->event();
    if (hipEventRecord(b, s) == hipSuccess) t_prof->record(name, work, a, b);
}

Plan::~Plan() {
    clear_graphs(*this);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) {
        (void)hipStreamSynchronize(side);
        (void)hipStreamDestroy(side);
    }
    if (side2) {
        (void)hipStreamSynchronize(side2);
        (void)hipStreamDestroy(side2);
    }
    if (ev_ready) (void)hipEventDestroy(ev_ready);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (ev_ready2) (void)hipEventDestroy(ev_ready2);
    if (ev_done2) (void)hipEventDestroy(ev_done2);
    if (h_row_ptr) (void)hipHostFree(h_row_ptr);
    if (h_col_idx) (void)hipHostFree(h_col_idx);
    if (h_perm) (void)hipHostFree(h_perm);
    if (h_flags) (void)hipHostFree(h_flags);
    if (h_scalars) (void)hipHostFree(h_scalars);
}

}  // namespace hs
