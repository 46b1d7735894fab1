// Device-side helpers shared by the HIP translation units (wave64, 256-thread blocks).
#pragma once

#include <mutex>

#include "hs_internal.h"

namespace hs {

constexpr int NT = 256;          // threads per workgroup (4 waves)
constexpr int WAVE = 64;

// Global-memory pointers with an explicit address space. Pointers read from task tables
// are otherwise generic, and the compiler emits flat accesses for them; a flat load also
// counts against the LDS wait counter, so every LDS read in a loop would wait for all
// outstanding global loads. Hot loops access global memory through HS_G pointers.
#define HS_G __attribute__((address_space(1)))
template <class T> __device__ inline HS_G T* gp(T* p) { return (HS_G T*)p; }
template <class T> __device__ inline const HS_G T* gp(const T* p) { return (const HS_G T*)p; }

// Raise the dynamic LDS limit of a kernel once per process (safe from several host threads)
inline void set_lds_limit(std::once_flag& flag, const void* kernel, size_t bytes) {
    std::call_once(flag, [&] {
        HS_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)));
    });
}

inline void check_launch(const char* name) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw Error{HSOLVE_ERR_DEVICE, std::string("launch of ") + name + ": " + hipGetErrorString(e)};
}

__device__ inline double wave_sum(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ inline float wave_sum(float v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ inline double wave_max(double v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Orders the memory accesses of the lanes of one wave around divergent code (a result that
// one lane wrote to LDS is read by the others afterwards).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
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

__device__ inline double block_max(double v, double* red) {
    v = wave_max(v);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < NT / WAVE; ++i) s = fmax(s, red[i]);
    return s;
}

}  // namespace hs
