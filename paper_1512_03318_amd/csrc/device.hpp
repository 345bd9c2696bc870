// Device helpers shared by the kernels (GEMMs of every precision, casts, Lanczos).
#pragma once

#include "internal.hpp"

namespace mrd {

// Device pointers read from a table in device memory are generic to the compiler, which
// then emits flat loads; those also count on the LDS counter, so every wait on them
// waits for all loads in flight.  Typed as global memory they become global loads with
// per-load waits.
#define MRD_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MRD_GLOBAL T* glb(T* p) {
  return (MRD_GLOBAL T*)p;
}

template <typename T>
struct Cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cplx<T> ldc(const T* base, int64_t off) {
  // one complex element = two consecutive reals
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v = *reinterpret_cast<const v2*>(base + 2 * off);
  return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void stc(T* base, int64_t off, T re, T im) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = re;
  v.y = im;
  *reinterpret_cast<v2*>(base + 2 * off) = v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b on XCD b % 8); give
// each XCD a contiguous run of the tile list, so tiles of one output sector (which share
// operand panels) meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Sums the K-split partial tiles (tm x tn each) of one output tile in split order and
// stores it.  Block (x, y): output tile x, elements [1024 y, 1024 y + 1024) of the tile.
// REAL: real partial tiles and result (tm x tn values at the start of each slot).
template <typename T, int FLAGS, typename Prob = GemmProb, bool REAL = false>
__global__ void __launch_bounds__(256) gemm_split_reduce_kernel(const Prob* __restrict__ probs,
                                                                const GemmTile* __restrict__ tiles,
                                                                const int64_t* __restrict__ rows,
                                                                const T* __restrict__ part,
                                                                T* __restrict__ C, int tm, int tn,
                                                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const GemmTile tile = tiles[blockIdx.x];
  const Prob P = probs[tile.prob];
  const int tiles_n = (P.N + tn - 1) / tn;
  const int64_t slot = (int64_t)tm * tn;
  const int64_t base = (int64_t)P.slot0 + ((int64_t)tile.tm * tiles_n + tile.tn) * P.nks;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = blockIdx.y * 1024 + q * 256 + threadIdx.x;
    if (e >= tm * tn) break;
    const int r = e / tn, c = e - r * tn;
    const int i = tile.tm * tm + r, j = tile.tn * tn + c;
    if (i >= P.M || j >= P.N) continue;
    // the partials of this element (at most 8 splits) are all loaded before they are
    // summed, in split order
    T pr[8], pi[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      pr[ks] = 0;
      pi[ks] = 0;
      if (ks < P.nks) {
        if constexpr (REAL) {
          pr[ks] = part[2 * (base + ks) * slot + e];
        } else {
          const Cplx<T> v = ldc(part, (base + ks) * slot + e);
          pr[ks] = v.re;
          pi[ks] = v.im;
        }
      }
    }
    T re = 0, im = 0;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
      if (ks < P.nks) {
        re += pr[ks];
        im += pi[ks];
      }
    const int64_t rb = (FLAGS & G_C_ROWMAP) ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
    if constexpr (REAL) {
      if (FLAGS & G_C_F64) reinterpret_cast<double*>(C)[rb + j] = (double)re;
      else C[rb + j] = re;
    }
    else if (FLAGS & G_C_F64) stc(reinterpret_cast<double*>(C), rb + j, (double)re, (double)im);
    else stc(C, rb + j, re, im);
  }
}

}  // namespace mrd
