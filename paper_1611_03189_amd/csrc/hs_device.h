// Device-side helpers shared by the HIP translation units (wave64, 256-thread blocks).
#pragma once

#include <mutex>

#include "hs_internal.h"

namespace hs {

constexpr int NT = 256;          // threads per workgroup (4 waves) unless a kernel states another count
constexpr int WAVE = 64;

// Global-memory pointers with an explicit address space. Pointers read from task tables
// are otherwise generic, and the compiler emits flat accesses for them; a flat load also
// counts against the LDS wait counter, so every LDS read in a loop would wait for all
// outstanding global loads. Hot loops access global memory through HS_G pointers.
#define HS_G __attribute__((address_space(1)))
template <class T> __device__ inline HS_G T* gp(T* p) { return (HS_G T*)p; }
template <class T> __device__ inline const HS_G T* gp(const T* p) { return (const HS_G T*)p; }
// Read-only view of global memory that no thread of the running kernel writes: loads at
// wave-uniform addresses through it become scalar loads (the scalar cache starts every
// dispatch clean). Used only for such reads.
#define HS_C __attribute__((address_space(4)))
template <class T> __device__ inline const HS_C T* cp(const T* p) { return (const HS_C T*)p; }

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

// operand / accumulator type of v_mfma_f64_16x16x4f64
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core product per wave in the storage type T: lane l supplies
// A(l % 16, l / 16) and B(l / 16, l % 16); result register r holds C(row(l, r), l % 16). The
// FP64 and FP32 instructions take the same operand lanes but place their result rows
// differently (measured on gfx950).
template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef dbl4 acc;
    __device__ static acc zero() { return dbl4{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc mac(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
};
template <> struct Mma<float> {
    typedef flt4 acc;
    __device__ static acc zero() { return flt4{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc mac(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

// Wave-wide reductions with DPP: two quad permutations and two rotations by 4 and 8 leave
// every lane with the total of its row of 16; two row broadcasts (lane 15 into rows 1 and 3,
// lane 31 into rows 2 and 3) gather the four rows in lane 63, which is read back as a
// uniform value, so every lane returns the same, bitwise identical result.
template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_move(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_move(float v, float fill) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), CTRL, ROWS, 0xF, false));
}

__device__ inline double lane63(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), WAVE - 1);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), WAVE - 1);
    return __hiloint2double(hi, lo);
}

__device__ inline float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), WAVE - 1));
}

constexpr int DPP_QUAD_1032 = 0xB1, DPP_QUAD_2301 = 0x4E, DPP_ROR4 = 0x124, DPP_ROR8 = 0x128,
              DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143;

// Sum over the 16 lanes of each DPP row, the same bits in every lane: a butterfly whose
// partners swap equal partial sums (pairs, quads, then the halves of the row by mirroring),
// so each addition is the same pair of operands in either order.
// (Every lane's source is inside its row, so the moves need no fill value.)
template <int CTRL>
__device__ inline double dpp_row_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ inline double row16_sum(double v) {
    v += dpp_row_move<DPP_QUAD_1032>(v);
    v += dpp_row_move<DPP_QUAD_2301>(v);
    v += dpp_row_move<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_row_move<DPP_ROW_MIRROR>(v);
    return v;
}

template <class T>
__device__ inline T wave_sum(T v) {
    v += dpp_move<DPP_QUAD_1032>(v, T(0));
    v += dpp_move<DPP_QUAD_2301>(v, T(0));
    v += dpp_move<DPP_ROR4>(v, T(0));
    v += dpp_move<DPP_ROR8>(v, T(0));
    v += dpp_move<DPP_BCAST15, 0xA>(v, T(0));
    v += dpp_move<DPP_BCAST31, 0xC>(v, T(0));
    return lane63(v);
}

__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_move<DPP_QUAD_1032>(v, v));
    v = fmax(v, dpp_move<DPP_QUAD_2301>(v, v));
    v = fmax(v, dpp_move<DPP_ROR4>(v, v));
    v = fmax(v, dpp_move<DPP_ROR8>(v, v));
    v = fmax(v, dpp_move<DPP_BCAST15, 0xA>(v, v));
    v = fmax(v, dpp_move<DPP_BCAST31, 0xC>(v, v));
    return lane63(v);
}

// dst(i, c) = f(src(i, c), i, c) over a rows x cols column-major block by the whole
// workgroup: consecutive threads take consecutive elements (coalesced), and each thread
// issues eight loads before its stores, so the copy is not bound by one load's latency.
template <int NTH = NT, class PD, class PS, class F>
__device__ inline void copy_block(PD dst, size_t ldd, PS src, size_t lds, int rows, int cols, F f) {
    const int total = rows * cols;
    if (total <= 0) return;
    const int dq = NTH / rows, dr = NTH % rows;
    int e = threadIdx.x, i = e % rows, c = e / rows;
    auto step = [&]() {
        i += dr;
        c += dq;
        if (i >= rows) {
            i -= rows;
            ++c;
        }
    };
    for (; e + 7 * NTH < total; e += 8 * NTH) {
        int ii[8], cc[8];
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            ii[u] = i;
            cc[u] = c;
            v[u] = src[i + size_t(c) * lds];
            step();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[ii[u] + size_t(cc[u]) * ldd] = f(v[u], ii[u], cc[u]);
    }
    for (; e < total; e += NTH) {
        dst[i + size_t(c) * ldd] = f(src[i + size_t(c) * lds], i, c);
        step();
    }
}

template <int NTH = NT, class PD, class PS>
__device__ inline void copy_block(PD dst, size_t ldd, PS src, size_t lds, int rows, int cols) {
    copy_block<NTH>(dst, ldd, src, lds, rows, cols, [](double x, int, int) { return x; });
}

// Orders the memory accesses of the lanes of one wave around divergent code (a result that
// one lane wrote to LDS is read by the others afterwards).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// block-wide sum over NTH threads; `red` must hold NTH/WAVE doubles; result valid in every thread
template <int NTH = NT>
__device__ inline double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NTH / WAVE; ++i) s += red[i];
    return s;
}

template <int NTH = NT>
__device__ inline double block_max(double v, double* red) {
    v = wave_max(v);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < NTH / WAVE; ++i) s = fmax(s, red[i]);
    return s;
}

}  // namespace hs
