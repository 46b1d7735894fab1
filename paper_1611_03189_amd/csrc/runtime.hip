// Device memory pools, pinned staging of task tables, plan teardown.
#include <algorithm>

#include "hs_internal.h"

namespace hs {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Pool::~Pool() { release(); }

void* Pool::alloc(size_t bytes) {
    bytes = align256(bytes ? bytes : 1);
    while (cur_ < chunks_.size() && off_ + bytes > chunks_[cur_].size) {
        used_before_ += off_;
        ++cur_;
        off_ = 0;
    }
    if (cur_ == chunks_.size()) {
        size_t sz = bytes > chunk_ ? bytes : chunk_;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error{HSOLVE_ERR_OOM, "device allocation of " + std::to_string(sz) + " bytes failed"};
        }
        chunks_.push_back({static_cast<char*>(p), sz});
        off_ = 0;
    }
    void* p = chunks_[cur_].p + off_;
    off_ += bytes;
    size_t used = used_before_ + off_;
    if (used > high_) high_ = used;
    return p;
}

size_t Pool::in_use() const { return used_before_ + off_; }

size_t Pool::reserved() const {
    size_t s = 0;
    for (const auto& c : chunks_) s += c.size;
    return s;
}

void Pool::reset() {
    cur_ = 0;
    off_ = 0;
    used_before_ = 0;
}

void Pool::release() {
    for (auto& c : chunks_) (void)hipFree(c.p);
    chunks_.clear();
    reset();
    high_ = 0;
}

Staging::~Staging() {
    if (host_) (void)hipHostFree(host_);
}

void* Staging::upload(const void* src, size_t bytes, Pool& dst_pool, hipStream_t s) {
    size_t need = align256(bytes);
    if (off_ + need > cap_) {
        // Growing would move memory that queued copies may still read: callers reset the
        // staging only after a synchronisation, so a fresh, larger buffer is safe to use
        // once the stream has drained.
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
    void* d = dst_pool.alloc(bytes);
    HS_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
    return d;
}

// First GPU use of a plan: device copies of the pattern and of the leaf order.
void upload_pattern(Plan& P) {
    if (P.d_row_ptr) return;
    const int n = P.n;
    HS_HIP(hipMalloc(&P.d_row_ptr, sizeof(int64_t) * (n + 1)));
    HS_HIP(hipMalloc(&P.d_col_idx, sizeof(int32_t) * std::max<int64_t>(1, P.nnz)));
    HS_HIP(hipMalloc(&P.d_values, sizeof(double) * std::max<int64_t>(1, P.nnz)));
    HS_HIP(hipMalloc(&P.d_perm, sizeof(int32_t) * 2 * n));
    HS_HIP(hipMalloc(&P.d_pos_super, sizeof(int32_t) * n));
    P.d_iperm = P.d_perm + n;
    std::vector<int32_t> pos_super(n, 0);
    if (P.L > 0)
        for (int i = 0; i < (1 << P.L); ++i)
            for (int q = P.leaf_off[i]; q < P.leaf_off[i + 1]; ++q) pos_super[q] = i >> 1;
    HS_HIP(hipMemcpy(P.d_row_ptr, P.row_ptr.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    if (P.nnz)
        HS_HIP(hipMemcpy(P.d_col_idx, P.col_idx.data(), sizeof(int32_t) * P.nnz, hipMemcpyHostToDevice));
    HS_HIP(hipMemcpy(P.d_perm, P.perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HS_HIP(hipMemcpy(P.d_iperm, P.iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
    HS_HIP(hipMemcpy(P.d_pos_super, pos_super.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
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
    if (side) {
        (void)hipStreamSynchronize(side);
        (void)hipStreamDestroy(side);
    }
    if (ev_ready) (void)hipEventDestroy(ev_ready);
    if (ev_done) (void)hipEventDestroy(ev_done);
    if (d_row_ptr) (void)hipFree(d_row_ptr);
    if (d_col_idx) (void)hipFree(d_col_idx);
    if (d_values) (void)hipFree(d_values);
    if (d_perm) (void)hipFree(d_perm);
    if (d_pos_super) (void)hipFree(d_pos_super);
    if (h_scalars) (void)hipHostFree(h_scalars);
}

}  // namespace hs
