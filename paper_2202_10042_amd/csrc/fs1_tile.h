// fs1_tile.h -- the wave-interleaved tile layout of the solve vectors.
//
// During the iterations of the fused and general paths the scaling vectors
// and the marginal copies are kept in a wave-interleaved layout: the 64 runs
// of R entries of a wavefront form a tile of 64 R entries in which entry j of
// lane i's run sits at  tile + (j / V) 64 V + i V + j % V  (V entries per 16
// bytes).  The k-th 16-byte load or store of every lane then covers one
// contiguous kilobyte (per-thread runs would touch every 64-byte segment four
// times, once per instruction), while each thread still holds its own run.
// The tile of run `run` starts at entry (run - lane) R.
#pragma once

#include "fs1_device.h"

namespace fs1 {

template <typename T, int R>
__device__ __forceinline__ void tile_load(const T* __restrict__ p, int64_t run, int lane,
                                          T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  static_assert(R % V == 0, "runs are whole 16-byte vectors");
  using VT = typename Vec16<T>::type;
  const VT* q = reinterpret_cast<const VT*>(p + (run - lane) * R) + lane;
#pragma unroll
  for (int i = 0; i < R / V; ++i) {
    const VT v = q[i * kWave];
    if constexpr (V == 2) {
      x[2 * i] = v.x;
      x[2 * i + 1] = v.y;
    } else {
      x[4 * i] = v.x;
      x[4 * i + 1] = v.y;
      x[4 * i + 2] = v.z;
      x[4 * i + 3] = v.w;
    }
  }
}

// Non-temporal stores of a run in the tile layout: the lines are not left
// dirty in the XCD's L2 for the write-back at the end of the kernel (the
// fused path's new vectors; 3.9% per iteration at N = 2^20 in binary64).
template <typename T, int R>
__device__ __forceinline__ void tile_store_nt(T* __restrict__ p, int64_t run, int lane,
                                              const T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  static_assert(R % V == 0, "runs are whole 16-byte vectors");
  T* q = p + (run - lane) * R + lane * V;
#pragma unroll
  for (int i = 0; i < R / V; ++i)
#pragma unroll
    for (int u = 0; u < V; ++u) __builtin_nontemporal_store(x[i * V + u], q + i * kWave * V + u);
}

template <typename T, int R>
__device__ __forceinline__ void tile_store(T* __restrict__ p, int64_t run, int lane,
                                           const T (&x)[R]) {
  constexpr int V = Vec16<T>::n;
  static_assert(R % V == 0, "runs are whole 16-byte vectors");
  using VT = typename Vec16<T>::type;
  VT* q = reinterpret_cast<VT*>(p + (run - lane) * R) + lane;
#pragma unroll
  for (int i = 0; i < R / V; ++i) {
    VT v;
    if constexpr (V == 2) {
      v.x = x[2 * i];
      v.y = x[2 * i + 1];
    } else {
      v.x = x[4 * i];
      v.y = x[4 * i + 1];
      v.z = x[4 * i + 2];
      v.w = x[4 * i + 3];
    }
    q[i * kWave] = v;
  }
}

// In-place change of layout of a vector of whole chunks (runs -> tiles or
// back).  A wave's tile holds exactly the wave's runs, and the barrier makes
// every load of the workgroup complete before any store.
template <typename T, int R, bool TO_TILES>
__global__ __launch_bounds__(kBlock) void k_relayout(T* v) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t run = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  T x[R];
  if constexpr (TO_TILES) {
    load_run_z<T, R>(v, run * R, x);
  } else {
    tile_load<T, R>(v, run, lane, x);
  }
  __syncthreads();
  if constexpr (TO_TILES) {
    tile_store<T, R>(v, run, lane, x);
  } else {
    store_run_z<T, R>(v, run * R, x);
  }
}

}  // namespace fs1
