// Device helpers of the operator kernels: mortar side maps, division by a small point count,
// volume indexing, table lookup and the XCD-aware workgroup order.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace hpdg {
namespace {

constexpr int kFaces = 6;

// how the mortar's point grid maps onto one side's face axes (a, b)
struct Map {
  int swap, flipA, flipB, halfA, halfB;
};

// l / q through the 16.16 reciprocal qinv = ceil(65536 / q) (no integer division): exact for
// 0 <= l < 1024 and 1 <= q <= 20
__device__ inline int qdiv(int l, int qinv) { return (l * qinv) >> 16; }

// volume index of the node with index k along axis d and (i, j) along the face axes t0 < t1
// (arithmetic only: indexed private arrays would live in scratch memory)
__device__ inline int vidx(int n, int d, int t0, int t1, int k, int i, int j) {
  const int s0 = t0 == 0 ? 1 : n;            // t0 is axis 0 or 1
  const int s1 = t1 == 1 ? n : n * n;        // t1 is axis 1 or 2
  const int sd = d == 0 ? 1 : (d == 1 ? n : n * n);
  return k * sd + i * s0 + j * s1;
}

template <typename T>
__device__ inline const T* tab(const LevelView<T>& L, int kind, int n, int q) {
  return L.tab + L.tv.off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q];
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b on XCD b % 8), each with
// its own L2.  Remap so that every XCD walks one contiguous range of the element list: elements
// that are neighbours in the (Morton-ordered) list then meet in the same L2, where the face
// layers and the shared mortar metric they both read are reused.  A bijection of [0, G).
__device__ inline unsigned xcd_remap(unsigned b, unsigned G) {
  constexpr unsigned X = 8;
  const unsigned q = G / X, r = G % X, x = b % X, i = b / X;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

}  // namespace
}  // namespace hpdg
