// Packed symmetric element-block mat-vec shared by the block-Jacobi kernel and the fused
// apply + block-Jacobi Chebyshev step: device helpers only.
//
// Storage of one N x N symmetric block: its lower triangle in 64-row panels; panel r0 (rows
// r0 .. r0 + m - 1, m = min(64, N - r0)) starts at r0 (r0 + 1) / 2 and holds the full columns
// 0 .. r0 - 1 (m entries each, column-major), then its diagonal tile's columns j = 0 .. m - 1,
// each holding rows j .. m - 1.
#pragma once
#include <hip/hip_runtime.h>

namespace hpdg {

namespace {

// ---- the packed mat-vec ----
// The lower triangle is visited by column blocks of G columns; in a block, by the 64-row panels
// at and below it: the diagonal panel's tile (tile columns j0 .. j0 + G - 1 of its diagonal
// tile) and then the full columns c0 .. c0 + G - 1 of every lower panel. The column part is
// accumulated per lane across the panels and reduced over the wave once per column block.
constexpr int kGroup = 16;

// G per-lane values w[t] (partial sums of columns c0 + t) summed over the wave; returns, in
// every lane, the total of column c0 + (lane % G): halving exchange steps (each lane keeps the
// half selected by one lane bit, adding its partner's copy of that half), then all-reduce
// steps over the lane groups of G. The order of additions is fixed.
template <int G, typename T>
__device__ __forceinline__ T wave_column_sums(T (&w)[G], int lane) {
#pragma unroll
  for (int step = 0; (G >> (step + 1)) >= 1; ++step) {  // an affine counter, so that it unrolls
    const int s = G >> (step + 1);
    const bool hi = (lane & s) != 0;
#pragma unroll
    for (int k = 0; k < s; ++k) {
      // both halves are exchanged and the select acts on the sums: a select between two array
      // elements would be turned into a per-lane array index (a chain of selects over w)
      const T lo = w[k] + __shfl_xor(w[k], s, 64);
      const T up = w[k + s] + __shfl_xor(w[k + s], s, 64);
      w[k] = hi ? up : lo;
    }
  }
  T v = w[0];
#pragma unroll
  for (int s = G; s < 64; s *= 2) v += __shfl_xor(v, s, 64);
  return v;
}

// the G values of columns c0 .. c0 + G - 1 in the rows of panel r0 (lane l: row r0 + l). Every
// lane loads: lanes outside the panel or the triangle read a clamped address inside the same
// column and their value is discarded later, so that no load sits behind a per-lane branch.
template <int G, typename S, typename T>
__device__ __forceinline__ void load_tile(const S* Pe, int N, int c0, int r0, int lane, T (&v)[G]) {
  const int m = min(64, N - r0);
  const S* Pp = Pe + (long long)r0 * (r0 + 1) / 2;
  if (c0 < r0) {  // full columns (c0 + G <= r0: c0 and r0 are multiples of G and 64)
    const S* q = Pp + (long long)c0 * m + min(lane, m - 1);
#pragma unroll
    for (int t = 0; t < G; ++t) v[t] = T(q[t * m]);
  } else {  // diagonal tile columns j0 .. j0 + G - 1 (column j holds rows j .. m - 1)
    const S* Pd = Pp + (long long)r0 * m;
    const int j0 = c0 - r0;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const int j = min(j0 + t, m - 1);
      const int st = j * m - j * (j - 1) / 2;
      v[t] = T(Pd[st + min(max(lane - j, 0), m - 1 - j)]);
    }
  }
}

// one tile: lane l adds its row's products to z[r0 + l] (LDS, index i only touched by lane
// i % 64) and its column partials (times r[r0 + l]) to w; the diagonal entry counts once
template <int G, typename T>
__device__ __forceinline__ void tile_products(int N, int c0, int r0, int lane, const T* rs, T* zs, T (&w)[G],
                                              const T (&v)[G]) {
  const int m = min(64, N - r0);
  const bool act = lane < m;
  const T xr = act ? rs[r0 + lane] : T(0);
  T acc = 0;
  if (c0 < r0) {
    // lanes past the panel hold finite entries of the same column (clamped loads): their acc
    // is never stored and their xr is 0, so their products need no mask
#pragma unroll
    for (int t = 0; t < G; ++t) {
      acc += v[t] * rs[c0 + t];
      w[t] += v[t] * xr;
    }
  } else {
    const int j0 = c0 - r0;
#pragma unroll
    for (int t = 0; t < G; ++t) {
      const int j = j0 + t;
      const bool in = act && j < m && lane >= j;
      const T vv = in ? v[t] : T(0);
      acc += vv * rs[r0 + min(j, m - 1)];
      w[t] += lane > j ? vv * xr : T(0);
    }
  }
  if (act) zs[r0 + lane] += acc;
}

// this wave's part of z = Binv r for one element: the column blocks kb = wv, wv + waves, ... of the
// packed block Pe (N rows) applied to r (rs, LDS); accumulated into zs (N entries of LDS owned by
// this wave, zeroed by the caller; index i is only touched by lane i % 64). wv must be uniform
// over the wave (a scalar register), so that the loop control and block addresses stay scalar.
template <typename S, typename T>
__device__ __forceinline__ void packed_block_partial(const S* Pe, int N, const T* rs, T* zs, int waves, int wv,
                                                     int lane) {
  constexpr int G = kGroup;
#pragma unroll 1
  for (int kb = wv; kb * G < N; kb += waves) {
    const int c0 = kb * G;  // a multiple of G by construction (lets the compiler simplify the indexing)
    T w[G];
#pragma unroll
    for (int t = 0; t < G; ++t) w[t] = 0;
#pragma unroll 1
    for (int r0 = c0 & ~63; r0 < N; r0 += 64) {
      T v[G];
      load_tile<G>(Pe, N, c0, r0, lane, v);
      tile_products<G>(N, c0, r0, lane, rs, zs, w, v);
    }
    const T cs = wave_column_sums<G>(w, lane);
    // lane == (c0 + lane % G) % 64 owns that index
    if (lane / G == ((c0 / G) & (64 / G - 1)) && c0 + (lane & (G - 1)) < N) zs[c0 + (lane & (G - 1))] += cs;
  }
}

}  // namespace

}  // namespace hpdg
