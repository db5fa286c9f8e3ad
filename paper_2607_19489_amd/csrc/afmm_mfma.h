// MFMA helpers shared by the forward and adjoint kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace afmm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T> struct Acc4;
template <> struct Acc4<float> { typedef f32x4 type; };
template <> struct Acc4<double> { typedef f64x4 type; };

// D[16x16] += A[16x4] B[4x16]; lane l holds A[l%16][l/16] and B[l/16][l%16].
// Accumulator element r of lane l is D[acc_row(l/16, r)][l%16]: rows 4(l/16)+r
// for FP32 and (l/16)+4r for FP64 (checked on gfx950 by a lane-layout probe).
__device__ inline f32x4 mfma16(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline f64x4 mfma16(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <typename T>
__device__ inline int acc_row(int krow, int r) { return sizeof(T) == 4 ? 4 * krow + r : krow + 4 * r; }

// Device pointers read out of tables in memory reach the compiler as generic
// pointers, and loads through them become flat loads, which count against the
// LDS wait counter as well: every wait for an LDS read would then also wait
// for all global loads in flight (the next tap's prefetch).  Such pointers
// always address global memory; the kernels load and store through these.
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
template <typename T> using gmut = __attribute__((address_space(1))) T*;
template <typename T> __device__ inline gptr<T> as_global(const T* p) { return (gptr<T>)p; }
template <typename T> __device__ inline gmut<T> as_global_mut(T* p) { return (gmut<T>)p; }

// Orders the LDS accesses of one wave: writes before the call are visible to
// every lane of the same wave after it (no block barrier needed when each
// wave only touches its own LDS slice).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte vectors
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// XCD-aware tile order: consecutive blocks land on different XCDs, so block b
// takes tile (b % 8) * ceil(n/8) + b / 8 and each XCD sweeps one contiguous
// (spatially compact) range of tiles.
__device__ inline int xcd_tile(int ntiles) {
  const int per = (ntiles + 7) / 8;
  return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}

// D~ rows of one source offset staged in LDS: sD[o * KS + g] = D~_g at child
// offset o (g < K; zeros up to KS), then one zero slot at 8 KS, copied from
// rows already in that layout and padded to whole 16-byte vectors (SDP values
// per offset): NTH threads, thread t takes vectors t, t + NTH, ...
template <typename T, int SDP, int NTH>
__device__ inline void load_dstage_t(int di, const T* __restrict__ Dst, typename Vec16<T>::type* vD) {
  using V = typename Vec16<T>::type;
  constexpr int NV = SDP / (16 / (int)sizeof(T)), NJ = (NV + NTH - 1) / NTH;
  gptr<V> src = (gptr<V>)as_global(Dst + (size_t)di * SDP);
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    if (NV % NTH == 0 || t + NTH * j < NV) vD[j] = src[t + NTH * j];
}

template <typename T, int SDP, int NTH>
__device__ inline void store_dstage_t(T* sD, const typename Vec16<T>::type* vD) {
  using V = typename Vec16<T>::type;
  constexpr int NV = SDP / (16 / (int)sizeof(T)), NJ = (NV + NTH - 1) / NTH;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    if (NV % NTH == 0 || t + NTH * j < NV) ((V*)sD)[t + NTH * j] = vD[j];
}

}  // namespace afmm
