// gfx950 operator kernel of the hpdg library: y = A x on one multigrid level.
//
// One workgroup per element computes y_e = (A x)_e completely, so every output is written
// once, without atomics, and the result is bitwise reproducible:
//   * volume: the stiffness term by sum factorisation through the GL points
//     (Eq. harald-stiff): three 1-D passes to the GL points, the reference gradient by the
//     GL collocation derivative, the metric contraction G (Eq. stiffness-3, with w J and k
//     folded in), and the transposed passes back to the LGL test functions;
//   * faces: the SIPG terms of Eq. lh2 on every mortar of the element (Eq. temp-E), both
//     sides' traces interpolated onto the mortar's GL points through the hp projections of
//     Fig. mortar (1-D matrices for the sub-face halves and the degree change), the flux
//     formed for the own side only and lifted back through the transposed interpolation.
//     The six faces are processed together, one mortar per face per round (a face of a
//     coarse element facing four finer elements takes four rounds).
// Each mortar is therefore evaluated once from each side.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "apply_common.hpp"
#include "blocks.hpp"
#include "device.hpp"

namespace hpdg {

namespace {

// threads per workgroup (one element per workgroup)
#ifndef HPDG_APPLY_THREADS
#define HPDG_APPLY_THREADS 256
#endif
constexpr int kThreads = HPDG_APPLY_THREADS;
// compact: kernels of a fixed degree with at most two volume nodes per thread; the element's
// coefficients sit at the start of the shared region (dead once the volume phase has read
// them: the face phases take both sides' traces from the trace buffer) and each thread keeps
// its volume results in registers, so the workgroup needs less LDS
struct Layout {
  int NM, QM, QMM;
  bool compact;
  size_t fixed, vol, ra, rb, y, tasks;
  __host__ __device__ Layout(int nm, int qm, int qmm, bool cmp = false) : NM(nm), QM(qm), QMM(qmm), compact(cmp) {
    const size_t n3 = size_t(NM) * NM * NM;
    fixed = (compact ? 0 : 2 * n3) + size_t(QM) * NM + size_t(QM) * QM + QM + 2 * NM;
    const size_t tsz = size_t(NM) * QM * (NM > QM ? NM : QM);
    vol = (compact ? n3 : 0) + 4 * size_t(QM) * QM * QM + 2 * tsz;
    if (compact) {  // fused face phases: RA holds T1, then S; RB the traces, then the fluxes
      ra = kFaces * mx3(6 * size_t(NM) * QMM, 3 * size_t(QMM) * NM, 0);
      rb = kFaces * mx3(4 * size_t(NM) * NM, 4 * size_t(QMM) * QMM, 0);
    } else {  // large enough for both face paths
      ra = kFaces * mx3(size_t(NM) * NM * NM, 6 * size_t(NM) * QMM, 4 * size_t(QMM) * QMM);
      rb = kFaces * mx3(4 * size_t(NM) * NM, 8 * size_t(QMM) * QMM, 3 * size_t(QMM) * NM);
    }
    y = 2 * kFaces * size_t(NM) * NM;
    tasks = (kFaces * sizeof(Task) + 15) / 16 * 16;
  }
  __host__ __device__ static size_t mx3(size_t a, size_t b, size_t c) {
    return a > b ? (a > c ? a : c) : (b > c ? b : c);
  }
  // the face phases also stage the six 1-D mortar matrices of a uniform level
  __host__ __device__ size_t faces() const { return ra + rb + y + 6 * size_t(QMM) * NM; }
  __host__ __device__ size_t region() const { return vol > faces() ? vol : faces(); }
  __host__ __device__ size_t bytes(size_t scalar) const { return tasks + scalar * (fixed + region()); }
};

// The Jacobi-scaled Chebyshev step behind a fused apply: region[0 .. n^3) holds r = b - A x of
// element e (the face buffers are free by then). z = M^-1 r (the packed block over the
// workgroup's waves, partial z per wave after r; or z = dinv r), p and x are updated, and with
// bs.trace_out the face traces of the new x are written as trace_kernel writes them. NC: n
// when fixed at compile time, else 0.
template <typename T, int NC>
__device__ void fused_step_tail(int n_rt, const ElemInfo& I, long long e, T* region, const T* dfo, int NM,
                                const BlockStep<T>& bs) {
  const int N = NC ? NC : n_rt, N2 = N * N, N3 = N2 * N;
  constexpr int kWaves = kThreads >= 64 ? kThreads / 64 : 1;  // the launcher requires whole waves
  const T* rs = region;
  const int lane = int(threadIdx.x & 63);
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  T* zs = region + N3 + wv * N3;
  if (!bs.dinv) {
    for (int i = lane; i < N3; i += 64) zs[i] = 0;
    __syncthreads();
    packed_block_partial<T, T>(bs.P + bs.poff[e], N3, rs, zs, kWaves, wv, lane);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N3; i += kThreads) {
    T z = 0;
    if (bs.dinv) {
      z = bs.dinv[I.off + i] * rs[i];
    } else {
#pragma unroll
      for (int k = 0; k < kWaves; ++k) z += rs[N3 + k * N3 + i];
    }
    const T pn = bs.first ? bs.alpha * z : bs.alpha * z + bs.beta * bs.p[I.off + i];
    bs.p[I.off + i] = pn;
    const T xn = bs.x[I.off + i] + pn;
    bs.x[I.off + i] = xn;
    region[i] = xn;  // r is no longer read (each thread reads only its own partials after it)
  }
  if (bs.trace_out) {
    // the next step's traces (as trace_kernel): values on each face and the reference normal
    // derivative there
    __syncthreads();
    for (int g = threadIdx.x; g < 12 * N2; g += kThreads) {
      const int f = g / (2 * N2), r = g % (2 * N2), li = r % N2;
      const int d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      const int i = li % N, j = li / N;
      T v;
      if (r < N2) {
        v = region[vidx(N, d, t0, t1, (f & 1) ? N - 1 : 0, i, j)];
      } else {
        v = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) v += dfo[(f & 1) * NM + k] * region[vidx(N, d, t0, t1, k, i, j)];
      }
      bs.trace_out[I.toff + g] = v;
    }
  }
}

// Face terms of a level whose elements all have N nodes and whose mortars all have Q GL
// points per axis (uniform degree): every size is a compile-time constant, the six 1-D
// matrices (values / derivatives at the full, lower-half and upper-half point sets) are
// staged in LDS once, and each phase maps threads to (task, item) with constant strides.
// Adds the face terms to sy and writes y (FUSE: runs the Jacobi-scaled Chebyshev step bs on
// the result instead, in the same workgroup).
template <typename T, int N, int Q, bool COMPACT, bool FUSE>
__device__ void faces_uniform(const LevelView<T>& L, const ElemInfo& I, long long e, T* __restrict__ y,
                              const T* sy, const T (&syr)[2], const T* dfo, T* region, Task* tasks,
                              const Layout& lay, const BlockStep<T>& bs) {
  constexpr int N2 = N * N, N3 = N2 * N, QQ = Q * Q, NQ = N * Q;
  const int NM = lay.NM, QMM = lay.QMM;
  const int raS = int(lay.ra / kFaces), rbS = int(lay.rb / kFaces);
  T* mats = region;  // [kind 0..5][Q][N]
  // RB: traces (4 NM^2), then the flux coefficients (4 QMM^2); RA: first-pass values of both
  // sides (6 NM QMM), then the first transposed pass (3 QMM NM)
  T* RA = mats + 6 * QMM * NM;
  T* RB = RA + lay.ra;
  T* Yf = RB + lay.rb;
  T* Yn = Yf + kFaces * NM * NM;
  for (int i = threadIdx.x; i < 6 * NQ; i += blockDim.x) mats[i] = tab(L, i / NQ, N, Q)[i % NQ];
  for (int i = threadIdx.x; i < 2 * kFaces * NM * NM; i += blockDim.x) Yf[i] = 0;
  int rounds = 0;
#pragma unroll
  for (int f = 0; f < kFaces; ++f) rounds = I.fcnt[f] > rounds ? I.fcnt[f] : rounds;
  for (int r = 0; r < rounds; ++r) {
    for (int f = threadIdx.x; f < kFaces; f += blockDim.x) tasks[f] = make_task(L, e, f, r);
    __syncthreads();
    // P1: traces (values, reference normal derivative) of both sides from the trace buffer
    for (int g = threadIdx.x; g < kFaces * 2 * N2; g += blockDim.x) {
      const int t = g / (2 * N2), li = g % (2 * N2);
      const Task& tk = tasks[t];
      if (!tk.valid) continue;
      const bool own = li < N2;
      if (!own && !tk.other) continue;
      const int l2 = own ? li : li - N2;
      const long long off = own ? I.toff + 2LL * tk.f * N2 : tk.ooff;
      T* tr = RB + t * rbS + (own ? 0 : 2 * NM * NM);
      tr[l2] = L.trace[off + l2];
      tr[NM * NM + l2] = L.trace[off + N2 + l2];
    }
    __syncthreads();
    // P2: first interpolation pass (along face axis a): u, du/da, du/dn
    for (int g = threadIdx.x; g < kFaces * 2 * NQ; g += blockDim.x) {
      const int t = g / (2 * NQ), li = g % (2 * NQ);
      const Task& tk = tasks[t];
      if (!tk.valid) continue;
      const bool own = li < NQ;
      if (!own && !tk.other) continue;
      const int l2 = own ? li : li - NQ;
      const Map m = own ? tk.me : tk.ot;
      const T* F = RB + t * rbS + (own ? 0 : 2 * NM * NM);
      const T* Nd = F + NM * NM;
      const T* Ma = mats + (2 * m.halfA) * NQ;
      const T* Da = Ma + NQ;
      const int xg = l2 % Q, j = l2 / Q;
      const int ra = m.flipA ? Q - 1 - xg : xg;
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T fv = F[j * N + i], ma = Ma[ra * N + i];
        s0 += ma * fv;
        s1 += Da[ra * N + i] * fv;
        s2 += ma * Nd[j * N + i];
      }
      T* T1 = RA + t * raS + (own ? 0 : 3 * NM * QMM);
      T1[j * Q + xg] = s0;
      T1[NM * QMM + j * Q + xg] = s1;
      T1[2 * NM * QMM + j * Q + xg] = s2;
    }
    __syncthreads();
    // P3+P4: second pass (along face axis b) of both sides at one mortar point: u, du/da,
    // du/db, du/dn; then the SIPG flux there (own side, own frame) into RB
    for (int g = threadIdx.x; g < kFaces * QQ; g += blockDim.x) {
      const int t = g / QQ, li = g % QQ;
      const Task& tk = tasks[t];
      if (!tk.valid) continue;
      // side values at the point with index l2 of that side's frame
      auto at_point = [&](bool own, int l2, T& v0, T& v1, T& v2, T& v3) {
        const Map m = own ? tk.me : tk.ot;
        const T* T1 = RA + t * raS + (own ? 0 : 3 * NM * QMM);
        const T* Mb = mats + (2 * m.halfB) * NQ;
        const T* Db = Mb + NQ;
        const int xg = l2 % Q, yg = l2 / Q;
        const int rb = m.flipB ? Q - 1 - yg : yg;
        T g0 = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const T mb = Mb[rb * N + j];
          const T a0 = T1[j * Q + xg];
          g0 += mb * a0;
          g1 += mb * T1[NM * QMM + j * Q + xg];
          g2 += Db[rb * N + j] * a0;
          g3 += mb * T1[2 * NM * QMM + j * Q + xg];
        }
        v0 = g0;
        v1 = g1;
        v2 = g2;
        v3 = g3;
      };
      const int side = tk.side;
      const int npts = tk.gmode ? QQ : 1;
      const T* mg = L.mgeo + tk.geo;
      const int f = tk.f, d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      const int xg = li % Q, yg = li / Q;
      const int cc = tk.me.swap ? yg : xg, dd = tk.me.swap ? xg : yg;
      const int pp = tk.gmode ? cc + Q * dd : 0;
      T wS;
      if (tk.gmode) {
        wS = mg[6 * npts + pp];
      } else {
        const T* wm = L.tab + L.tv.w_off[Q];
        wS = wm[cc] * wm[dd] * mg[6];
      }
      const T sig = mg[7 * npts + pp];
      const T ma = mg[(3 * side + t0) * npts + pp];
      const T mb = mg[(3 * side + t1) * npts + pp];
      const T mn = mg[(3 * side + d) * npts + pp];
      T u_me, ga, gb, gn;
      at_point(true, li, u_me, ga, gb, gn);
      const T g_me = ma * ga + mb * gb + mn * gn;
      T Af, Bc;
      if (tk.interior) {
        T u_o = 0, g_o = 0;
        if (tk.other) {
          const int os = 1 - side, od = tk.of >> 1;
          const int ot0 = od == 0 ? 1 : 0, ot1 = od == 2 ? 1 : 2;
          const int oi = tk.ot.swap ? dd + Q * cc : cc + Q * dd;
          T oa, ob, on;
          at_point(false, oi, u_o, oa, ob, on);
          g_o = mg[(3 * os + ot0) * npts + pp] * oa + mg[(3 * os + ot1) * npts + pp] * ob +
                mg[(3 * os + od) * npts + pp] * on;
        }
        const T jmp = u_me - u_o;
        Af = wS * (sig * jmp - T(0.5) * (g_me - g_o));
        Bc = T(-0.5) * wS * jmp;
      } else {
        Af = wS * (sig * u_me - g_me);
        Bc = -wS * u_me;
      }
      T* CF = RB + t * rbS;
      CF[li] = Af;
      CF[QMM * QMM + li] = Bc * ma;
      CF[2 * QMM * QMM + li] = Bc * mb;
      CF[3 * QMM * QMM + li] = Bc * mn;
    }
    __syncthreads();
    // P5: first transposed pass (along the own face axis a)
    for (int g = threadIdx.x; g < kFaces * NQ; g += blockDim.x) {
      const int t = g / NQ, li = g % NQ;
      const Task& tk = tasks[t];
      if (!tk.valid) continue;
      const T* Ma = mats + (2 * tk.me.halfA) * NQ;
      const T* Da = Ma + NQ;
      const T* CF = RB + t * rbS;
      const int i = li % N, yg = li / N;
      T s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int xg = 0; xg < Q; ++xg) {
        const int ra = tk.me.flipA ? Q - 1 - xg : xg;
        const T ma = Ma[ra * N + i];
        const int gi = yg * Q + xg;
        s1 += ma * CF[gi] + Da[ra * N + i] * CF[QMM * QMM + gi];
        s2 += ma * CF[2 * QMM * QMM + gi];
        s3 += ma * CF[3 * QMM * QMM + gi];
      }
      T* S = RA + t * raS;
      S[li] = s1;
      S[QMM * NM + li] = s2;
      S[2 * QMM * NM + li] = s3;
    }
    __syncthreads();
    // P6: second transposed pass (along b) into the per-face sums
    for (int g = threadIdx.x; g < kFaces * N2; g += blockDim.x) {
      const int t = g / N2, li = g % N2;
      const Task& tk = tasks[t];
      if (!tk.valid) continue;
      const T* Mb = mats + (2 * tk.me.halfB) * NQ;
      const T* Db = Mb + NQ;
      const T* S = RA + t * raS;
      const int i = li % N, j = li / N;
      T yf = 0, yn = 0;
#pragma unroll
      for (int yg = 0; yg < Q; ++yg) {
        const int rb = tk.me.flipB ? Q - 1 - yg : yg;
        const T mb = Mb[rb * N + j];
        yf += mb * S[yg * N + i] + Db[rb * N + j] * S[QMM * NM + yg * N + i];
        yn += mb * S[2 * QMM * NM + yg * N + i];
      }
      Yf[tk.f * NM * NM + li] += yf;
      Yn[tk.f * NM * NM + li] += yn;
    }
    __syncthreads();
  }
  // face sums -> element
  auto finish = [&](int idx, T acc) {
    const int c0 = idx % N, c1 = (idx / N) % N, c2 = idx / N2;
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
      if (I.fcnt[f] == 0) continue;
      const int d = f >> 1;
      const int kd = d == 0 ? c0 : (d == 1 ? c1 : c2);
      const int li = d == 0 ? c2 * N + c1 : (d == 1 ? c2 * N + c0 : c1 * N + c0);
      acc += dfo[(f & 1) * NM + kd] * Yn[f * NM * NM + li];
      if (kd == ((f & 1) ? N - 1 : 0)) acc += Yf[f * NM * NM + li];
    }
    if constexpr (FUSE)
      region[idx] = bs.b[I.off + idx] - acc;  // r = b - A x (the face buffers before Yf are free now)
    else
      y[I.off + idx] = acc;
  };
  if constexpr (COMPACT) {  // node threadIdx.x + it kThreads of this thread
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (int(threadIdx.x) + it * kThreads < N3) finish(int(threadIdx.x) + it * kThreads, syr[it]);
  } else {
    for (int idx = threadIdx.x; idx < N3; idx += blockDim.x) finish(idx, sy[idx]);
  }
  if constexpr (FUSE) fused_step_tail<T, N>(N, I, e, region, dfo, NM, bs);
}

// NT, QT > 0: element degree + 1 and volume GL points fixed at compile time (the bucket's
// elements); 0: read from the element record.  UNI: uniform-degree level (faces_uniform).
template <typename T, int NT, int QT, bool UNI, bool FUSE = false>
__global__ void __launch_bounds__(kThreads) apply_kernel(LevelView<T> L, const int* __restrict__ elems,
                                                         long long count, const T* x, T* __restrict__ y,
                                                         BlockStep<T> bs) {
  extern __shared__ unsigned char smem_raw[];
  if ((long long)blockIdx.x >= count) return;
  const unsigned bid = xcd_remap(blockIdx.x, gridDim.x);  // gridDim.x == count
  const long long e = elems ? elems[bid] : (long long)bid;
  const ElemInfo I = L.einfo[e];
  const int n = NT ? NT : I.n, q = QT ? QT : I.q;
  const int n2 = n * n, n3 = n2 * n, q3 = q * q * q;
  constexpr bool COMPACT = NT > 0 && NT * NT * NT <= 2 * kThreads;
  static_assert(!FUSE || UNI, "the fused smoother step runs on one-degree levels");
  const Layout lay(L.nmax, L.qmax, L.qmmax, COMPACT);
  const int NM = lay.NM, QM = lay.QM, QMM = lay.QMM;

  Task* tasks = reinterpret_cast<Task*>(smem_raw);
  T* p = reinterpret_cast<T*>(smem_raw + lay.tasks);
  T* su = p;
  T* sy = p + NM * NM * NM;
  if (!COMPACT) p += 2 * NM * NM * NM;
  T* Bm = p; p += QM * NM;        // LGL -> GL interpolation [q][n]
  T* Dg = p; p += QM * QM;        // GL collocation derivative [q][q]
  T* w = p; p += QM;              // GL weights
  T* dfo = p; p += 2 * NM;        // l_k'(-1), l_k'(+1) of the own basis
  T* region = p;
  if (COMPACT) {
    su = region;  // the coefficients open the region; the volume buffers follow
    sy = nullptr;
  }
  T* A0 = region + (COMPACT ? NM * NM * NM : 0);
  T* A1 = A0 + QM * QM * QM;
  T* A2 = A1 + QM * QM * QM;
  T* A3 = A2 + QM * QM * QM;
  const int tsz = NM * QM * (NM > QM ? NM : QM);
  T* tA = A3 + QM * QM * QM;
  T* tB = tA + tsz;
  // face phases (alias the volume buffers): ping-pong regions RA / RB and the face sums
  T* RA = region;
  T* RB = RA + lay.ra;
  T* Yf = RB + lay.rb;
  T* Yn = Yf + kFaces * NM * NM;
  const int raS = int(lay.ra / kFaces), rbS = int(lay.rb / kFaces);

  {
    const T* B = tab(L, 0, n, q);
    const T* Dgg = L.tab + L.tv.dg_off[q];
    const T* wg = L.tab + L.tv.w_off[q];
    const T* dfg = L.tab + L.tv.dface_off[n];
    for (int i = threadIdx.x; i < n3; i += blockDim.x) su[i] = x[I.off + i];
    for (int i = threadIdx.x; i < q * n; i += blockDim.x) Bm[i] = B[i];
    for (int i = threadIdx.x; i < q * q; i += blockDim.x) Dg[i] = Dgg[i];
    for (int i = threadIdx.x; i < q; i += blockDim.x) w[i] = wg[i];
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) dfo[(i / n) * NM + i % n] = dfg[i];
  }
  __syncthreads();

  // ---- volume: u -> GL values (three 1-D passes) ----
  for (int idx = threadIdx.x; idx < n2 * q; idx += blockDim.x) {
    const int a = idx % q, kj = idx / q;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < n; ++i) acc += Bm[a * n + i] * su[kj * n + i];
    tA[idx] = acc;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, k = idx / (q * q);
    T acc = 0;
#pragma unroll
    for (int j = 0; j < n; ++j) acc += Bm[b * n + j] * tA[(k * n + j) * q + a];
    tB[idx] = acc;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int ba = idx % (q * q), c = idx / (q * q);
    T acc = 0;
#pragma unroll
    for (int k = 0; k < n; ++k) acc += Bm[c * n + k] * tB[k * q * q + ba];
    A0[idx] = acc;  // [c][b][a]
  }
  __syncthreads();
  // ---- reference gradient at the GL points and the metric contraction ----
  const T* G = L.vgeo + I.vgeo;
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int t = 0; t < q; ++t) {
      g0 += Dg[a * q + t] * A0[(c * q + b) * q + t];
      g1 += Dg[b * q + t] * A0[(c * q + t) * q + a];
      g2 += Dg[c * q + t] * A0[(t * q + b) * q + a];
    }
    T G00, G01, G02, G11, G12, G22;
    if (I.vmode == 0) {
      const T ww = w[a] * w[b] * w[c];
      G00 = G[0] * ww; G01 = G[1] * ww; G02 = G[2] * ww;
      G11 = G[3] * ww; G12 = G[4] * ww; G22 = G[5] * ww;
    } else {
      G00 = G[idx]; G01 = G[q3 + idx]; G02 = G[2 * q3 + idx];
      G11 = G[3 * q3 + idx]; G12 = G[4 * q3 + idx]; G22 = G[5 * q3 + idx];
    }
    A1[idx] = G00 * g0 + G01 * g1 + G02 * g2;
    A2[idx] = G01 * g0 + G11 * g1 + G12 * g2;
    A3[idx] = G02 * g0 + G12 * g1 + G22 * g2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    T r = 0;
#pragma unroll
    for (int t = 0; t < q; ++t) {
      r += Dg[t * q + a] * A1[(c * q + b) * q + t];
      r += Dg[t * q + b] * A2[(c * q + t) * q + a];
      r += Dg[t * q + c] * A3[(t * q + b) * q + a];
    }
    if (I.mass && L.mcoef) r += L.mcoef[I.mq + idx] * A0[idx];
    A0[idx] = r;
  }
  __syncthreads();
  // ---- back to the LGL test functions (transposed passes) ----
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int ba = idx % (q * q), k = idx / (q * q);
    T acc = 0;
#pragma unroll
    for (int c = 0; c < q; ++c) acc += Bm[c * n + k] * A0[c * q * q + ba];
    tB[idx] = acc;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n2 * q; idx += blockDim.x) {
    const int a = idx % q, j = (idx / q) % n, k = idx / (n * q);
    T acc = 0;
#pragma unroll
    for (int b = 0; b < q; ++b) acc += Bm[b * n + j] * tB[(k * q + b) * q + a];
    tA[idx] = acc;  // [k][j][a]
  }
  __syncthreads();
  // COMPACT: this thread's volume results (nodes threadIdx.x and threadIdx.x + kThreads)
  T syr[2] = {0, 0};
  auto back_a = [&](int idx) {
    const int i = idx % n, kj = idx / n;
    T acc = 0;
#pragma unroll
    for (int a = 0; a < q; ++a) acc += Bm[a * n + i] * tA[kj * q + a];
    return acc;
  };
  if constexpr (COMPACT) {
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (int(threadIdx.x) + it * kThreads < n3) syr[it] = back_a(int(threadIdx.x) + it * kThreads);
  } else {
    for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) sy[idx] = back_a(idx);
  }
  __syncthreads();  // the face phases reuse the volume buffers

  // ---- faces ----
  if constexpr (UNI) {
    faces_uniform<T, NT, QT, COMPACT, FUSE>(L, I, e, y, sy, syr, dfo, region, tasks, lay, bs);
    return;
  }
  int rounds = 0;
#pragma unroll
  for (int f = 0; f < kFaces; ++f) rounds = I.fcnt[f] > rounds ? I.fcnt[f] : rounds;
  for (int i = threadIdx.x; i < 2 * kFaces * NM * NM; i += blockDim.x) Yf[i] = 0;  // Yf and Yn
  for (int r = 0; r < rounds; ++r) {
    for (int f = threadIdx.x; f < kFaces; f += blockDim.x) tasks[f] = make_task(L, e, f, r);
    __syncthreads();
    // P1: traces (values and reference normal derivative) of both sides from the trace buffer
#define C1(t) (tasks[t].valid ? n2 + (tasks[t].other ? tasks[t].no * tasks[t].no : 0) : 0)
    for_items(HPDG_COUNTS(C1), [&](int t, int li) {
      const Task& tk = tasks[t];
      T* tr = RB + t * rbS;  // Fm, Nm, Fo, No at strides NM^2
      if (li < n2) {
        const long long off = I.toff + 2LL * tk.f * n2;
        tr[li] = L.trace[off + li];
        tr[NM * NM + li] = L.trace[off + n2 + li];
      } else {
        const int lo = li - n2, no2 = tk.no * tk.no;
        tr[2 * NM * NM + lo] = L.trace[tk.ooff + lo];
        tr[3 * NM * NM + lo] = L.trace[tk.ooff + no2 + lo];
      }
    });
    __syncthreads();
    // P2: first interpolation pass (along face axis a) of u, du/da, du/dn, both sides
#define C2(t) (tasks[t].valid ? tasks[t].qm * (n + (tasks[t].other ? tasks[t].no : 0)) : 0)
    for_items(HPDG_COUNTS(C2), [&](int t, int li) {
      const Task& tk = tasks[t];
      const int qm = tk.qm;
      const bool own = li < n * qm;
      const int ns = own ? n : tk.no;
      const int l2 = own ? li : li - n * qm;
      const Map m = own ? tk.me : tk.ot;
      const T* F = RB + t * rbS + (own ? 0 : 2 * NM * NM);
      const T* N = F + NM * NM;
      const T* Ma = L.tab + (own ? tk.meA : tk.otA);
      const T* Da = L.tab + (own ? tk.meAd : tk.otAd);
      const int j = qdiv(l2, tk.qinv), xg = l2 - j * qm;
      const int ra = m.flipA ? qm - 1 - xg : xg;
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll 4
      for (int i = 0; i < ns; ++i) {
        const T fv = F[j * ns + i], ma = Ma[ra * ns + i];
        s0 += ma * fv;
        s1 += Da[ra * ns + i] * fv;
        s2 += ma * N[j * ns + i];
      }
      T* T1 = RA + t * raS + (own ? 0 : 3 * NM * QMM);
      T1[j * qm + xg] = s0;
      T1[NM * QMM + j * qm + xg] = s1;
      T1[2 * NM * QMM + j * qm + xg] = s2;
    });
    __syncthreads();
    // P3+P4: second pass (along face axis b) of both sides at one mortar point: u, du/da,
    // du/db, du/dn; then the SIPG flux there (own side, own frame) into RB
#define C4(t) (tasks[t].valid ? tasks[t].qm * tasks[t].qm : 0)
    for_items(HPDG_COUNTS(C4), [&](int t, int li) {
      const Task& tk = tasks[t];
      const int qm = tk.qm, qq = qm * qm, side = tk.side;
      // side values at the point with index l2 of that side's frame
      auto at_point = [&](bool own, int l2, T& v0, T& v1, T& v2, T& v3) {
        const int ns = own ? n : tk.no;
        const Map m = own ? tk.me : tk.ot;
        const T* T1 = RA + t * raS + (own ? 0 : 3 * NM * QMM);
        const T* Mb = L.tab + (own ? tk.meB : tk.otB);
        const T* Db = L.tab + (own ? tk.meBd : tk.otBd);
        const int yg = qdiv(l2, tk.qinv), xg = l2 - yg * qm;
        const int rb = m.flipB ? qm - 1 - yg : yg;
        T g0 = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll 4
        for (int j = 0; j < ns; ++j) {
          const T mb = Mb[rb * ns + j];
          const T a0 = T1[j * qm + xg];
          g0 += mb * a0;
          g1 += mb * T1[NM * QMM + j * qm + xg];
          g2 += Db[rb * ns + j] * a0;
          g3 += mb * T1[2 * NM * QMM + j * qm + xg];
        }
        v0 = g0;
        v1 = g1;
        v2 = g2;
        v3 = g3;
      };
      const int npts = tk.gmode ? qq : 1;
      const T* mg = L.mgeo + tk.geo;
      const int f = tk.f, d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      const int yg = qdiv(li, tk.qinv), xg = li - yg * qm;
      const int cc = tk.me.swap ? yg : xg, dd = tk.me.swap ? xg : yg;
      const int rho = cc + qm * dd, pp = tk.gmode ? rho : 0;
      T wS;
      if (tk.gmode) {
        wS = mg[6 * npts + pp];
      } else {
        const T* wm = L.tab + L.tv.w_off[qm];
        wS = wm[cc] * wm[dd] * mg[6];
      }
      const T sig = mg[7 * npts + pp];
      const T ma = mg[(3 * side + t0) * npts + pp];
      const T mb = mg[(3 * side + t1) * npts + pp];
      const T mn = mg[(3 * side + d) * npts + pp];
      T u_me, ga, gb, gn;
      at_point(true, li, u_me, ga, gb, gn);
      const T g_me = ma * ga + mb * gb + mn * gn;
      T Af, Bc;
      if (tk.interior) {
        T u_o = 0, g_o = 0;
        if (tk.other) {
          const int os = 1 - side, od = tk.of >> 1;
          const int ot0 = od == 0 ? 1 : 0, ot1 = od == 2 ? 1 : 2;
          const int xo = tk.ot.swap ? dd : cc, yo = tk.ot.swap ? cc : dd;
          T oa, ob, on;
          at_point(false, xo + qm * yo, u_o, oa, ob, on);
          g_o = mg[(3 * os + ot0) * npts + pp] * oa + mg[(3 * os + ot1) * npts + pp] * ob +
                mg[(3 * os + od) * npts + pp] * on;
        }
        const T jmp = u_me - u_o;
        Af = wS * (sig * jmp - T(0.5) * (g_me - g_o));
        Bc = T(-0.5) * wS * jmp;
      } else {
        Af = wS * (sig * u_me - g_me);
        Bc = -wS * u_me;
      }
      T* CF = RB + t * rbS;
      CF[li] = Af;
      CF[QMM * QMM + li] = Bc * ma;
      CF[2 * QMM * QMM + li] = Bc * mb;
      CF[3 * QMM * QMM + li] = Bc * mn;
    });
    __syncthreads();
    // P5: first transposed pass (along the own face axis a)
#define C5(t) (tasks[t].valid ? tasks[t].qm * n : 0)
    for_items(HPDG_COUNTS(C5), [&](int t, int li) {
      const Task& tk = tasks[t];
      const int qm = tk.qm;
      const T* Ma = L.tab + tk.meA;
      const T* Da = L.tab + tk.meAd;
      const T* CF = RB + t * rbS;
      const int i = li % n, yg = li / n;
      T s1 = 0, s2 = 0, s3 = 0;
#pragma unroll 4
      for (int xg = 0; xg < qm; ++xg) {
        const int ra = tk.me.flipA ? qm - 1 - xg : xg;
        const T ma = Ma[ra * n + i];
        const int g = yg * qm + xg;
        s1 += ma * CF[g] + Da[ra * n + i] * CF[QMM * QMM + g];
        s2 += ma * CF[2 * QMM * QMM + g];
        s3 += ma * CF[3 * QMM * QMM + g];
      }
      T* S = RA + t * raS;
      S[li] = s1;  // [y][i]
      S[QMM * NM + li] = s2;
      S[2 * QMM * NM + li] = s3;
    });
    __syncthreads();
    // P6: second transposed pass (along b) into the per-face sums
#define C6(t) (tasks[t].valid ? n2 : 0)
    for_items(HPDG_COUNTS(C6), [&](int t, int li) {
      const Task& tk = tasks[t];
      const int qm = tk.qm;
      const T* Mb = L.tab + tk.meB;
      const T* Db = L.tab + tk.meBd;
      const T* S = RA + t * raS;
      const int i = li % n, j = li / n;
      T yf = 0, yn = 0;
#pragma unroll 4
      for (int yg = 0; yg < qm; ++yg) {
        const int rb = tk.me.flipB ? qm - 1 - yg : yg;
        const T mb = Mb[rb * n + j];
        yf += mb * S[yg * n + i] + Db[rb * n + j] * S[QMM * NM + yg * n + i];
        yn += mb * S[2 * QMM * NM + yg * n + i];
      }
      Yf[tk.f * NM * NM + li] += yf;
      Yn[tk.f * NM * NM + li] += yn;
    });
    __syncthreads();
  }
  // face sums -> element: values on the face layer, normal-derivative part along the lines
#undef C1
#undef C2
#undef C4
#undef C5
#undef C6
  auto finish = [&](int idx, T acc) {
    const int c0 = idx % n, c1 = (idx / n) % n, c2 = idx / n2;
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
      if (I.fcnt[f] == 0) continue;
      const int d = f >> 1;
      // node index along the normal axis and its (t0, t1) position on the face
      const int kd = d == 0 ? c0 : (d == 1 ? c1 : c2);
      const int li = d == 0 ? c2 * n + c1 : (d == 1 ? c2 * n + c0 : c1 * n + c0);
      acc += dfo[(f & 1) * NM + kd] * Yn[f * NM * NM + li];
      if (kd == ((f & 1) ? n - 1 : 0)) acc += Yf[f * NM * NM + li];
    }
    y[I.off + idx] = acc;
  };
  if constexpr (COMPACT) {  // node threadIdx.x + it kThreads of this thread
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (int(threadIdx.x) + it * kThreads < n3) finish(int(threadIdx.x) + it * kThreads, syr[it]);
  } else {
    for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) finish(idx, sy[idx]);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) trace_kernel(LevelView<T> L, const T* __restrict__ x) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int n = I.n, n2 = n * n;
  const T* u = x + I.off;
  const T* dfg = L.tab + L.tv.dface_off[n];  // l_k'(-1), then l_k'(+1)
  for (int g = threadIdx.x; g < 12 * n2; g += blockDim.x) {
    const int f = g / (2 * n2), r = g % (2 * n2), li = r % n2;
    const int d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
    const int i = li % n, j = li / n;
    T v;
    if (r < n2) {
      v = u[vidx(n, d, t0, t1, (f & 1) ? n - 1 : 0, i, j)];
    } else {
      const T* df = dfg + ((f & 1) ? n : 0);
      v = 0;
      for (int k = 0; k < n; ++k) v += df[k] * u[vidx(n, d, t0, t1, k, i, j)];
    }
    L.trace[I.toff + g] = v;
  }
}

template <typename T, int N, int Q, bool UNI, bool FUSE = false>
void launch_fixed(const LevelView<T>& L, const int* elems, long long count, const T* x, T* y, size_t lds,
                  hipStream_t s, const BlockStep<T>& bs = BlockStep<T>{}) {
  hipLaunchKernelGGL((apply_kernel<T, N, Q, UNI, FUSE>), dim3(unsigned(count)), dim3(kThreads), lds, s, L, elems,
                     count, x, y, bs);
}

}  // namespace

size_t apply_lds_bytes(int NM, int QM, int QMM, size_t scalar, bool compact) {
  return Layout(NM, QM, QMM, compact).bytes(scalar);
}

template <typename T>
void launch_traces(const LevelView<T>& L, const T* x, hipStream_t s) {
  if (L.n_elem == 0) return;  // also with self_only: the uniform face path reads the own traces
  hipLaunchKernelGGL((trace_kernel<T>), dim3(unsigned(L.n_elem)), dim3(kThreads), 0, s, L, x);
}

template <typename T>
void launch_apply(const LevelView<T>& L, const T* x, T* y, hipStream_t s) {
  if (L.n_elem == 0) return;
  launch_traces<T>(L, x, s);
  const size_t lds = apply_lds_bytes(L.nmax, L.qmax, L.qmmax, sizeof(T), false);
  hipLaunchKernelGGL((apply_kernel<T, 0, 0, false>), dim3(unsigned(L.n_elem)), dim3(kThreads), lds, s, L,
                     (const int*)nullptr, L.n_elem, x, y, BlockStep<T>{});
}

template <typename T>
void launch_apply_bucket(const LevelView<T>& L, int n, int q, int uniform, const int* elems, long long count,
                         const T* x, T* y, hipStream_t s) {
  if (count == 0) return;
  const size_t lds = apply_lds_bytes(L.nmax, L.qmax, L.qmmax, sizeof(T), false);
  // the fixed-degree kernels of degree n with n^3 <= 2 kThreads use the compact layout
  const size_t lds_c = apply_lds_bytes(L.nmax, L.qmax, L.qmmax, sizeof(T), n * n * n <= 2 * kThreads);
#define HPDG_CASE(NN, QQ)                                                                      \
  if (n == NN && q == QQ)                                                                       \
    return uniform ? launch_fixed<T, NN, QQ, true>(L, elems, count, x, y, lds_c, s)             \
                   : launch_fixed<T, NN, QQ, false>(L, elems, count, x, y, lds_c, s);
  HPDG_CASE(2, 2) HPDG_CASE(2, 3) HPDG_CASE(3, 3) HPDG_CASE(3, 4) HPDG_CASE(4, 4) HPDG_CASE(4, 5)
  HPDG_CASE(5, 5) HPDG_CASE(5, 6) HPDG_CASE(6, 6) HPDG_CASE(6, 7) HPDG_CASE(7, 7) HPDG_CASE(7, 8)
  HPDG_CASE(8, 8) HPDG_CASE(8, 9)
#undef HPDG_CASE
  hipLaunchKernelGGL((apply_kernel<T, 0, 0, false>), dim3(unsigned(count)), dim3(kThreads), lds, s, L, elems,
                     count, x, y, BlockStep<T>{});
}

bool apply_block_fusable(int nmax, int qmax, int qmmax, int n, int q, int uniform) {
  // mixed-degree levels keep the separate kernels: fused per degree bucket they measured slower
  if (!uniform || n * n * n > 2 * kThreads || kThreads % 64 != 0 || n < 2 || n > 8 || q < n || q > n + 1)
    return false;
  const Layout lay(nmax, qmax, qmmax, true);
  // r and one partial z per wave in the face buffers before the face sums (RA, RB)
  return lay.ra + lay.rb >= (1LL + kThreads / 64) * n * n * n;
}

template <typename T>
void launch_apply_block_cheb(const LevelView<T>& L, int n, int q, int uniform, const int* elems, long long count,
                             const T* x, const BlockStep<T>& bs, hipStream_t s) {
  if (count == 0) return;
  if (!apply_block_fusable(L.nmax, L.qmax, L.qmmax, n, q, uniform))
    throw Error(-7, "fused smoother step: level of several degrees, or degree outside the compact layout");
  const size_t lds = apply_lds_bytes(L.nmax, L.qmax, L.qmmax, sizeof(T), true);
#define HPDG_CASE(NN, QQ) \
  if (n == NN && q == QQ) return launch_fixed<T, NN, QQ, true, true>(L, elems, count, x, nullptr, lds, s, bs);
  HPDG_CASE(2, 2) HPDG_CASE(2, 3) HPDG_CASE(3, 3) HPDG_CASE(3, 4) HPDG_CASE(4, 4) HPDG_CASE(4, 5)
  HPDG_CASE(5, 5) HPDG_CASE(5, 6) HPDG_CASE(6, 6) HPDG_CASE(6, 7) HPDG_CASE(7, 7) HPDG_CASE(7, 8)
  HPDG_CASE(8, 8) HPDG_CASE(8, 9)
#undef HPDG_CASE
  throw Error(-7, "fused block step: no kernel for this (n, q)");
}

template void launch_apply_block_cheb<double>(const LevelView<double>&, int, int, int, const int*, long long,
                                              const double*, const BlockStep<double>&, hipStream_t);
template void launch_apply_block_cheb<float>(const LevelView<float>&, int, int, int, const int*, long long,
                                             const float*, const BlockStep<float>&, hipStream_t);
template void launch_traces<double>(const LevelView<double>&, const double*, hipStream_t);
template void launch_traces<float>(const LevelView<float>&, const float*, hipStream_t);
template void launch_apply<double>(const LevelView<double>&, const double*, double*, hipStream_t);
template void launch_apply<float>(const LevelView<float>&, const float*, float*, hipStream_t);
// ---- face-trace scratch of the apply for callers that cannot allocate -------------------
// The traces live in this fixed device array (each GPU the library runs on holds its own copy
// until the process ends).  Host code never passes the array's name to a kernel: it uses the
// device address that hipGetSymbolAddress returns for the current device, kept per device.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per HIP device: the address of that device's copy
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

void init_noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < int(g_scratch_ptr.size()) && g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw Error(-6, std::string("hipGetSymbolAddress of the no-allocation scratch: ") + hipGetErrorString(e));
  if (device >= int(g_scratch_ptr.size())) g_scratch_ptr.resize(device + 1, nullptr);
  g_scratch_ptr[device] = ptr;
}

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < int(g_scratch_ptr.size()) ? g_scratch_ptr[device] : nullptr;
}

template void launch_apply_bucket<double>(const LevelView<double>&, int, int, int, const int*, long long,
                                          const double*, double*, hipStream_t);
template void launch_apply_bucket<float>(const LevelView<float>&, int, int, int, const int*, long long,
                                         const float*, float*, hipStream_t);

}  // namespace hpdg
