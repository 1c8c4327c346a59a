// Device helpers shared by the operator kernels (apply.hip, apply_wave.hip): mortar maps,
// per-face tasks, table lookup, the flattened item loop over six faces and the XCD-aware
// workgroup order.
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

__device__ inline Map mortar_map(const MortarInfo& M, int side) {
  Map s{0, 0, 0, 0, 0};
  if (side) {
    s.swap = M.orient & 1;
    s.flipA = (M.orient >> 1) & 1;
    s.flipB = (M.orient >> 2) & 1;
    s.halfA = M.sub < 0 ? 0 : 1 + (M.sub & 1);
    s.halfB = M.sub < 0 ? 0 : 1 + ((M.sub >> 1) & 1);
  }
  return s;
}

// one (face, mortar) pair of the element in the current round
struct Task {
  int valid, f, side, interior, other, qm, gmode, no, of;
  Map me, ot;
  long long ooff, geo;  // neighbour trace offset, mortar metric offset
  // offsets (in the 1-D table) of the mortar interpolation matrices [qm][n_side]: value and
  // derivative rows along the side's face axis a (its half for the h step) and along b, for
  // the own side (me*) and the neighbour (ot*)
  int meA, meAd, meB, meBd, otA, otAd, otB, otBd;
  int qinv;  // ceil(65536 / qm): l / qm = (l * qinv) >> 16 exactly for 0 <= l < 1024
};

// l / q and l % q for the mortar's point count q through its 16.16 reciprocal (no integer division)
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

// flattened loop over the items of the six tasks: cnt[t] items of task t
// (counts passed as scalars and the task found by unrolled compares, so that nothing is an
// indexed private array)
template <typename F>
__device__ inline void for_items(int c0, int c1, int c2, int c3, int c4, int c5, F&& body) {
  const int p1 = c0, p2 = p1 + c1, p3 = p2 + c2, p4 = p3 + c3, p5 = p4 + c4, total = p5 + c5;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    int t = 0, base = 0;
    if (g >= p1) { t = 1; base = p1; }
    if (g >= p2) { t = 2; base = p2; }
    if (g >= p3) { t = 3; base = p3; }
    if (g >= p4) { t = 4; base = p4; }
    if (g >= p5) { t = 5; base = p5; }
    body(t, g - base);
  }
}

#define HPDG_COUNTS(expr) expr(0), expr(1), expr(2), expr(3), expr(4), expr(5)

// Task metadata for face f in round r (shared by the face paths): one 32-byte record
template <typename T>
__device__ inline Task make_task(const LevelView<T>& L, long long e, int f, int r) {
  // (read through memory: indexing a private copy of the element record with a per-thread
  // face would place it in scratch)
  const ElemInfo& Ig = L.einfo[e];
  Task tk;
  tk.valid = r < Ig.fcnt[f];
  tk.f = f;
  tk.side = tk.interior = tk.other = tk.qm = tk.gmode = tk.no = tk.of = 0;
  tk.me = tk.ot = Map{0, 0, 0, 0, 0};
  tk.ooff = tk.geo = 0;
  tk.meA = tk.meAd = tk.meB = tk.meBd = tk.otA = tk.otAd = tk.otB = tk.otBd = 0;
  tk.qinv = 1;
  if (tk.valid) {
    const FaceTask F = L.ftask[Ig.fstart[f] + r];
    tk.side = F.side;
    tk.interior = F.interior;
    tk.other = F.interior && !L.self_only;
    tk.qm = F.qm;
    tk.gmode = F.gmode;
    tk.geo = F.geo;
    tk.of = F.of;
    auto unpack = [](unsigned m) { return Map{int(m & 1), int((m >> 1) & 1), int((m >> 2) & 1), int((m >> 3) & 3), int((m >> 5) & 3)}; };
    tk.me = unpack(F.me);
    tk.ot = unpack(F.ot);
    if (tk.other) {
      tk.no = F.no;
      tk.ooff = F.ooff;
    }
    auto toff = [&](int kind, int n, int q) { return L.tv.off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q]; };
    const int qm = tk.qm, n = Ig.n;
    if (qm > 0) {
      tk.qinv = (65536 + qm - 1) / qm;
      tk.meA = toff(2 * tk.me.halfA, n, qm);
      tk.meAd = toff(1 + 2 * tk.me.halfA, n, qm);
      tk.meB = toff(2 * tk.me.halfB, n, qm);
      tk.meBd = toff(1 + 2 * tk.me.halfB, n, qm);
      if (tk.other) {
        tk.otA = toff(2 * tk.ot.halfA, tk.no, qm);
        tk.otAd = toff(1 + 2 * tk.ot.halfA, tk.no, qm);
        tk.otB = toff(2 * tk.ot.halfB, tk.no, qm);
        tk.otBd = toff(1 + 2 * tk.ot.halfB, tk.no, qm);
      }
    }
  }
  return tk;
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
