// gfx950 operator kernels of the hpdg library: y = A x on one multigrid level, in three launches.
//
//   1. trace_kernel: every element's face traces (the values at the n^2 LGL nodes of each face
//      and the reference normal derivative there).
//   2. mortar_kernel, one wavefront per mortar: the SIPG terms of Eq. lh2 on that mortar
//      (Eq. temp-E) for both of its sides at once.  Both sides' traces are interpolated onto the
//      mortar's GL points through the hp projections of Fig. mortar (1-D matrices for the
//      sub-face halves and the degree change), the flux is formed once per point (the value
//      flux of the two sides differs only in sign), and each side's part is lifted back through
//      its transposed interpolation onto its own face: n^2 values that multiply the test
//      functions' face values and n^2 that multiply their reference normal derivative, written
//      to that side's slot (one slot per entry of the element's face-mortar list).
//   3. apply_kernel, one workgroup per element: the stiffness term by sum factorisation through
//      the GL points (Eq. harald-stiff): three 1-D passes to the GL points, the reference
//      gradient by the GL collocation derivative, the metric contraction G (Eq. stiffness-3,
//      with w J and k folded in), the transposed passes back to the LGL test functions; then
//      the element's face slots are summed per face (list order) and added, and y_e is
//      stored once.
// Every output is written by exactly one workgroup, without atomics, in a fixed order of
// additions: the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "apply_common.hpp"
#include "blocks.hpp"
#include "device.hpp"

namespace hpdg {

namespace {

// threads per workgroup of the element kernel (one element per workgroup)
#ifndef HPDG_APPLY_THREADS
#define HPDG_APPLY_THREADS 256
#endif
constexpr int kThreads = HPDG_APPLY_THREADS;
constexpr int kWaves = kThreads >= 64 ? kThreads / 64 : 1;  // whole waves (checked by the launchers)

// LDS of the element kernel, in scalars, for at most NM LGL nodes and QM GL points per axis.
// compact: kernels of a fixed degree with at most two volume nodes per thread; the element's
// coefficients sit at the start of the shared region (dead once the volume phase has read them)
// and each thread keeps its volume results in registers.  After the volume phase the region
// holds the per-face sums of the face slots (12 NM^2) at ``ysum``; with the fused smoother
// step, r and one partial z per wave go first.
struct Layout {
  int NM, QM;
  bool compact;
  size_t fixed, vol, ysum, region;
  __host__ __device__ Layout(int nm, int qm, bool cmp, bool fuse) : NM(nm), QM(qm), compact(cmp) {
    const size_t n3 = size_t(NM) * NM * NM;
    fixed = (compact ? 0 : 2 * n3) + size_t(QM) * NM + size_t(QM) * QM + QM + 2 * NM;
    const size_t tsz = size_t(NM) * QM * (NM > QM ? NM : QM);
    vol = (compact ? n3 : 0) + 4 * size_t(QM) * QM * QM + 2 * tsz;
    ysum = fuse ? (1 + kWaves) * n3 : 0;
    const size_t faces = ysum + 12 * size_t(NM) * NM;
    region = vol > faces ? vol : faces;
  }
  __host__ __device__ size_t bytes(size_t scalar) const { return scalar * (fixed + region); }
};

// LDS of the mortar kernel, in scalars: both sides' traces (4 NM^2), later the flux
// coefficients (4 arrays of QMM^2 per side); the first interpolation pass of both sides
// (3 arrays of NM QMM per side), later the first transposed pass (as many)
__host__ __device__ inline size_t mortar_r1(int NM, int QMM) {
  const size_t a = 4 * size_t(NM) * NM, b = 8 * size_t(QMM) * QMM;
  return a > b ? a : b;
}
__host__ __device__ inline size_t mortar_lds_scalars(int NM, int QMM) {
  return mortar_r1(NM, QMM) + 6 * size_t(NM) * QMM;
}

// The Jacobi-scaled Chebyshev step behind a fused apply: region[0 .. n^3) holds r = b - A x of
// element e (the face buffers are free by then). z = M^-1 r (the packed block over the
// workgroup's waves, partial z per wave after r; or z = dinv r), p and x are updated, and with
// bs.trace_out the face traces of the new x are written as trace_kernel writes them. NC: n
// when fixed at compile time, else 0.
template <typename T, int NC>
__device__ void fused_step_tail(int n_rt, const ElemInfo& I, long long e, T* region, const T* dfo, int NM,
                                const BlockStep<T>& bs) {
  const int N = NC ? NC : n_rt, N2 = N * N, N3 = N2 * N;
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
    (bs.xo ? bs.xo : bs.x)[I.off + i] = xn;
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

// One wavefront per mortar.  Items of a phase are spread over the 64 lanes; every quantity
// of the mortar (degrees, rule, maps, matrix offsets) is the same in all lanes.  EST: instead
// of the SIPG terms, the mortar's part of the a posteriori estimator (Eqs. Eta2_Integrals):
// sum over its points of w S ((h_m / p_m) [[k grad u]]^2 + sigma [[u]]^2) inside, w S sigma
// (u - g_D)^2 on Dirichlet faces (w S, h_m and sigma of the estimator's grid), written to
// est.out at the mortar's index.
template <typename T, bool EST = false>
__global__ void __launch_bounds__(64) mortar_kernel(LevelView<T> L, long long count, EstFace est) {
  extern __shared__ unsigned char smem_raw[];
  if ((long long)blockIdx.x >= count) return;
  const long long mi = xcd_remap(blockIdx.x, gridDim.x);  // gridDim.x == count
  const MortarTask M = L.mtask[mi];
  const int NM = L.nmax, QMM = L.qmmax;
  const int lane = threadIdx.x;
  const int qm = M.q, qq = qm * qm;
  const int qinv = (65536 + qm - 1) / qm;
  const bool two = M.interior != 0;
  const bool other = two && !L.self_only;  // each side's flux sees the other side's trace
  const int n0 = M.n[0], n1 = two ? M.n[1] : 0;
  auto unpack = [](unsigned m) {
    return Map{int(m & 1), int((m >> 1) & 1), int((m >> 2) & 1), int((m >> 3) & 3), int((m >> 5) & 3)};
  };
  const Map m0 = unpack(M.map[0]), m1 = unpack(M.map[1]);
  auto toff = [&](int kind, int n) { return L.tv.off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + qm]; };
  // value and derivative rows [qm][n_s] along each side's face axes a and b (their halves)
  const T* A0 = L.tab + toff(2 * m0.halfA, n0);
  const T* A0d = L.tab + toff(1 + 2 * m0.halfA, n0);
  const T* B0 = L.tab + toff(2 * m0.halfB, n0);
  const T* B0d = L.tab + toff(1 + 2 * m0.halfB, n0);
  const T* A1 = two ? L.tab + toff(2 * m1.halfA, n1) : A0;
  const T* A1d = two ? L.tab + toff(1 + 2 * m1.halfA, n1) : A0d;
  const T* B1 = two ? L.tab + toff(2 * m1.halfB, n1) : B0;
  const T* B1d = two ? L.tab + toff(1 + 2 * m1.halfB, n1) : B0d;

  T* smem = reinterpret_cast<T*>(smem_raw);
  T* F = smem;                               // side s: values at F + 2 s NM^2, normal derivatives + NM^2
  T* CF = smem;                              // side s: 4 arrays of QMM^2 at CF + 4 s QMM^2
  T* T1 = smem + mortar_r1(NM, QMM);         // side s: 3 arrays of NM QMM at T1 + 3 s NM QMM
  T* S = T1;                                 // side s: 3 arrays of QMM NM (after T1 is read)
  const int NN = NM * NM, Q2 = QMM * QMM, NQ = NM * QMM;

  // P1: traces of both sides (2 n_s^2 contiguous scalars each)
  {
    const int c0 = 2 * n0 * n0, c1 = 2 * n1 * n1;
    for (int g = lane; g < c0 + c1; g += 64) {
      const bool s1 = g >= c0;
      const int l = s1 ? g - c0 : g, nsq = s1 ? n1 * n1 : n0 * n0;
      const int part = l >= nsq ? 1 : 0;
      F[(s1 ? 2 * NN : 0) + part * NN + (l - part * nsq)] = L.trace[(s1 ? M.tr[1] : M.tr[0]) + l];
    }
  }
  __syncthreads();
  // P2: first interpolation pass (along the side's face axis a) of u, du/da and du/dn
  {
    const int c0 = qm * n0, c1 = qm * n1;
    for (int g = lane; g < c0 + c1; g += 64) {
      const bool s1 = g >= c0;
      const int l2 = s1 ? g - c0 : g, ns = s1 ? n1 : n0;
      const Map mp = s1 ? m1 : m0;
      const T* Fs = F + (s1 ? 2 * NN : 0);
      const T* Ns = Fs + NN;
      const T* Ma = s1 ? A1 : A0;
      const T* Da = s1 ? A1d : A0d;
      const int j = qdiv(l2, qinv), xg = l2 - j * qm;
      const int ra = mp.flipA ? qm - 1 - xg : xg;
      T s0 = 0, sd = 0, sn = 0;
#pragma unroll 4
      for (int i = 0; i < ns; ++i) {
        const T fv = Fs[j * ns + i], ma = Ma[ra * ns + i];
        s0 += ma * fv;
        sd += Da[ra * ns + i] * fv;
        sn += ma * Ns[j * ns + i];
      }
      T* Ts = T1 + (s1 ? 3 * NQ : 0);
      Ts[j * qm + xg] = s0;
      Ts[NQ + j * qm + xg] = sd;
      Ts[2 * NQ + j * qm + xg] = sn;
    }
  }
  __syncthreads();
  // P3+P4: at each mortar point (cc, dd): both sides' u, du/da, du/db, du/dn (second pass
  // along b), the SIPG flux, and each side's coefficients in that side's frame into CF
  double eacc = 0;  // EST: this lane's points
  {
    const int npts = M.gmode ? qq : 1;
    const T* mg = L.mgeo + M.geo;
    const T* wm = L.tab + L.tv.w_off[qm];
    for (int g = lane; g < qq; g += 64) {
      const int dd = qdiv(g, qinv), cc = g - dd * qm;
      const int pp = M.gmode ? g : 0;
      const T wS = M.gmode ? mg[6 * npts + pp] : wm[cc] * wm[dd] * mg[6];
      const T sig = mg[7 * npts + pp];
      // side s at this point: index in its frame, its four values, its metric vector
      auto side_values = [&](int s, int& li, T& u, T& gr, T& ma, T& mb, T& mn) {
        const Map mp = s ? m1 : m0;
        const int ns = s ? n1 : n0;
        const int xg = mp.swap ? dd : cc, yg = mp.swap ? cc : dd;
        li = xg + qm * yg;
        const T* Ts = T1 + (s ? 3 * NQ : 0);
        const T* Mb = s ? B1 : B0;
        const T* Db = s ? B1d : B0d;
        const int rb = mp.flipB ? qm - 1 - yg : yg;
        T g0 = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll 4
        for (int j = 0; j < ns; ++j) {
          const T mbv = Mb[rb * ns + j];
          const T a0 = Ts[j * qm + xg];
          g0 += mbv * a0;
          g1 += mbv * Ts[NQ + j * qm + xg];
          g2 += Db[rb * ns + j] * a0;
          g3 += mbv * Ts[2 * NQ + j * qm + xg];
        }
        const int f = s ? M.f[1] : M.f[0], d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        ma = mg[(3 * s + t0) * npts + pp];
        mb = mg[(3 * s + t1) * npts + pp];
        mn = mg[(3 * s + d) * npts + pp];
        u = g0;
        gr = ma * g1 + mb * g2 + mn * g3;
      };
      int l0, l1 = 0;
      T u0, gr0, ma0, mb0, mn0, u1 = 0, gr1 = 0, ma1 = 0, mb1 = 0, mn1 = 0;
      side_values(0, l0, u0, gr0, ma0, mb0, mn0);
      if (two) side_values(1, l1, u1, gr1, ma1, mb1, mn1);
      if constexpr (EST) {
        // (h_m / p_m, g_D, S ratio, h_m ratio) at this point: w S and sigma of the grid the
        // integrals are taken on
        const double* ef = est.face + est.foff[mi] + 4 * g;
        const double w = double(wS) * ef[2], sg = double(sig) * ef[3];
        if (two) {
          const double J1 = double(gr0) + double(gr1), J2 = double(u0) - double(u1);
          eacc += w * (ef[0] * J1 * J1 + sg * J2 * J2);
        } else {
          const double J3 = double(u0) - ef[1];
          eacc += w * sg * J3 * J3;
        }
        continue;
      }
      T Af0, Bc0, Af1 = 0, Bc1 = 0;
      if (!two) {  // boundary: the Dirichlet form with zero data
        Af0 = wS * (sig * u0 - gr0);
        Bc0 = -wS * u0;
      } else if (other) {
        const T jmp = u0 - u1;
        Af0 = wS * (sig * jmp - T(0.5) * (gr0 - gr1));
        Bc0 = T(-0.5) * wS * jmp;
        Af1 = -Af0;
        Bc1 = -Bc0;
      } else {  // element-diagonal blocks: the other side's trace taken as zero
        Af0 = wS * (sig * u0 - T(0.5) * gr0);
        Bc0 = T(-0.5) * wS * u0;
        Af1 = wS * (sig * u1 - T(0.5) * gr1);
        Bc1 = T(-0.5) * wS * u1;
      }
      CF[l0] = Af0;
      CF[Q2 + l0] = Bc0 * ma0;
      CF[2 * Q2 + l0] = Bc0 * mb0;
      CF[3 * Q2 + l0] = Bc0 * mn0;
      if (two) {
        T* C1 = CF + 4 * Q2;
        C1[l1] = Af1;
        C1[Q2 + l1] = Bc1 * ma1;
        C1[2 * Q2 + l1] = Bc1 * mb1;
        C1[3 * Q2 + l1] = Bc1 * mn1;
      }
    }
  }
  if constexpr (EST) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) eacc += __shfl_xor(eacc, o, 64);
    if (lane == 0) est.out[est.tmortar[mi]] = eacc;
    return;
  }
  __syncthreads();
  // P5: first transposed pass (along the side's face axis a)
  {
    const int c0 = n0 * qm, c1 = n1 * qm;
    const int ninv0 = (65536 + n0 - 1) / n0, ninv1 = two ? (65536 + n1 - 1) / n1 : 1;
    for (int g = lane; g < c0 + c1; g += 64) {
      const bool s1 = g >= c0;
      const int li = s1 ? g - c0 : g, ns = s1 ? n1 : n0;
      const Map mp = s1 ? m1 : m0;
      const T* Ma = s1 ? A1 : A0;
      const T* Da = s1 ? A1d : A0d;
      const T* C = CF + (s1 ? 4 * Q2 : 0);
      const int yg = qdiv(li, s1 ? ninv1 : ninv0), i = li - yg * ns;
      T s1v = 0, s2v = 0, s3v = 0;
#pragma unroll 4
      for (int xg = 0; xg < qm; ++xg) {
        const int ra = mp.flipA ? qm - 1 - xg : xg;
        const T ma = Ma[ra * ns + i];
        const int p = yg * qm + xg;
        s1v += ma * C[p] + Da[ra * ns + i] * C[Q2 + p];
        s2v += ma * C[2 * Q2 + p];
        s3v += ma * C[3 * Q2 + p];
      }
      T* Ss = S + (s1 ? 3 * NQ : 0);
      Ss[li] = s1v;  // [yg][i]
      Ss[NQ + li] = s2v;
      Ss[2 * NQ + li] = s3v;
    }
  }
  __syncthreads();
  // P6: second transposed pass (along b) into each side's slot
  {
    const int c0 = n0 * n0, c1 = n1 * n1;
    const int ninv0 = (65536 + n0 - 1) / n0, ninv1 = two ? (65536 + n1 - 1) / n1 : 1;
    for (int g = lane; g < c0 + c1; g += 64) {
      const bool s1 = g >= c0;
      const int li = s1 ? g - c0 : g, ns = s1 ? n1 : n0;
      const Map mp = s1 ? m1 : m0;
      const T* Mb = s1 ? B1 : B0;
      const T* Db = s1 ? B1d : B0d;
      const T* Ss = S + (s1 ? 3 * NQ : 0);
      const int j = qdiv(li, s1 ? ninv1 : ninv0), i = li - j * ns;
      T yf = 0, yn = 0;
#pragma unroll 4
      for (int yg = 0; yg < qm; ++yg) {
        const int rb = mp.flipB ? qm - 1 - yg : yg;
        const T mbv = Mb[rb * ns + j];
        yf += mbv * Ss[yg * ns + i] + Db[rb * ns + j] * Ss[NQ + yg * ns + i];
        yn += mbv * Ss[2 * NQ + yg * ns + i];
      }
      T* out = L.slot + (s1 ? M.slot[1] : M.slot[0]);
      out[li] = yf;
      out[ns * ns + li] = yn;
    }
  }
}

// NT, QT > 0: element degree + 1 and volume GL points fixed at compile time (the bucket's
// elements), and the LDS laid out for them; 0: read from the element record, LDS for the
// level's largest.  FUSE: run the Jacobi-scaled Chebyshev step bs on the result instead of
// storing y.  The face slots of the element must be written (mortar_kernel) before the launch.
template <typename T, int NT, int QT, bool FUSE = false>
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
  static_assert(!FUSE || COMPACT, "the fused smoother step runs on the compact layout");
  const Layout lay(NT ? NT : L.nmax, QT ? QT : L.qmax, COMPACT, FUSE);
  const int NM = lay.NM, QM = lay.QM;

  T* p = reinterpret_cast<T*>(smem_raw);
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
  T* Ys = region + lay.ysum;  // after the volume phase: face f's value lift at f 2 n^2, normal lift + n^2

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
  __syncthreads();  // the face sums reuse the volume buffers

  // ---- faces: the element's slots, summed per face in list order ----
  {
    const ElemInfo& Ig = L.einfo[e];  // (read through memory: a per-thread face index into the
                                      // private copy would place it in scratch)
    const int f0 = I.fstart[0];
    for (int g = threadIdx.x; g < 12 * n2; g += blockDim.x) {
      const int f = g / (2 * n2), r2 = g - f * 2 * n2;
      const int cnt = Ig.fcnt[f];
      const T* sl = L.slot + I.soff + 2LL * (Ig.fstart[f] - f0) * n2 + r2;
      T acc = 0;
      for (int r = 0; r < cnt; ++r) acc += sl[2LL * r * n2];
      Ys[g] = acc;
    }
  }
  __syncthreads();
  // face sums -> element: values on the face layer, normal-derivative part along the lines
  auto finish = [&](int idx, T acc) {
    const int c0 = idx % n, c1 = (idx / n) % n, c2 = idx / n2;
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
      if (I.fcnt[f] == 0) continue;
      const int d = f >> 1;
      // node index along the normal axis and its (t0, t1) position on the face
      const int kd = d == 0 ? c0 : (d == 1 ? c1 : c2);
      const int li = d == 0 ? c2 * n + c1 : (d == 1 ? c2 * n + c0 : c1 * n + c0);
      acc += dfo[(f & 1) * NM + kd] * Ys[f * 2 * n2 + n2 + li];
      if (kd == ((f & 1) ? n - 1 : 0)) acc += Ys[f * 2 * n2 + li];
    }
    if constexpr (FUSE)
      region[idx] = bs.b[I.off + idx] - acc;  // r = b - A x (the face sums start after r and the partial z)
    else
      y[I.off + idx] = acc;
  };
  if constexpr (COMPACT) {  // node threadIdx.x + it kThreads of this thread
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (int(threadIdx.x) + it * kThreads < n3) finish(int(threadIdx.x) + it * kThreads, syr[it]);
  } else {
    for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) finish(idx, sy[idx]);
  }
  if constexpr (FUSE) fused_step_tail<T, NT>(NT, I, e, region, dfo, NM, bs);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) trace_kernel(LevelView<T> L, const T* __restrict__ x,
                                                         const int* __restrict__ list, long long count) {
  if ((long long)blockIdx.x >= count) return;
  const long long e = list ? list[blockIdx.x] : (long long)blockIdx.x;
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

template <typename T, int N, int Q, bool FUSE = false>
void launch_fixed(const LevelView<T>& L, const int* elems, long long count, const T* x, T* y, hipStream_t s,
                  const BlockStep<T>& bs = BlockStep<T>{}) {
  constexpr bool compact = N * N * N <= 2 * kThreads;
  const size_t lds = Layout(N, Q, compact, FUSE).bytes(sizeof(T));
  hipLaunchKernelGGL((apply_kernel<T, N, Q, FUSE>), dim3(unsigned(count)), dim3(kThreads), lds, s, L, elems, count,
                     x, y, bs);
}

template <typename T>
void launch_mortars(const LevelView<T>& L, hipStream_t s) {
  if (L.n_mtask == 0) return;
  const size_t lds = mortar_lds_scalars(L.nmax, L.qmmax) * sizeof(T);
  hipLaunchKernelGGL((mortar_kernel<T>), dim3(unsigned(L.n_mtask)), dim3(64), lds, s, L, L.n_mtask, EstFace{});
}

// ---- a posteriori estimator (Eqs. Eta2_Ingredients .. Eta2_Local), FP64 ------------------
// Volume part per element: h_e^2 p_e^2 sum over the volume GL points of W det J R^2 with
// R = g + (1 / det J) sum_d D_d F_d - c u, F_d = det J k (J^-1 J^-T grad_xi u)_d the
// contravariant flux at the GL points and D_d the GL collocation derivative along axis d.
__global__ void __launch_bounds__(kThreads) est_volume_kernel(LevelView<double> L, const double* __restrict__ x,
                                                              EstVolume ev, double* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[kThreads];
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int n = I.n, q = I.q, n3 = n * n * n, q3 = q * q * q;
  const int NM = L.nmax, QM = L.qmax;
  double* su = reinterpret_cast<double*>(smem_raw);
  double* tA = su + NM * NM * NM;
  double* tB = tA + NM * NM * QM;
  double* U = tB + NM * QM * QM;
  double* F0 = U + QM * QM * QM;
  double* F1 = F0 + QM * QM * QM;
  double* F2 = F1 + QM * QM * QM;
  const double* B = tab(L, 0, n, q);
  const double* Dg = L.tab + L.tv.dg_off[q];
  const double* w = L.tab + L.tv.w_off[q];
  for (int i = threadIdx.x; i < n3; i += blockDim.x) su[i] = x[I.off + i];
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n * q; idx += blockDim.x) {
    const int a = idx % q, kj = idx / q;
    double acc = 0;
    for (int i = 0; i < n; ++i) acc += B[a * n + i] * su[kj * n + i];
    tA[idx] = acc;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, k = idx / (q * q);
    double acc = 0;
    for (int j = 0; j < n; ++j) acc += B[b * n + j] * tA[(k * n + j) * q + a];
    tB[idx] = acc;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int ba = idx % (q * q), c = idx / (q * q);
    double acc = 0;
    for (int k = 0; k < n; ++k) acc += B[c * n + k] * tB[k * q * q + ba];
    U[idx] = acc;  // u at the GL points [c][b][a]
  }
  __syncthreads();
  const double* G = L.vgeo + I.vgeo;
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    double g0 = 0, g1 = 0, g2 = 0;
    for (int t = 0; t < q; ++t) {
      g0 += Dg[a * q + t] * U[(c * q + b) * q + t];
      g1 += Dg[b * q + t] * U[(c * q + t) * q + a];
      g2 += Dg[c * q + t] * U[(t * q + b) * q + a];
    }
    double G00, G01, G02, G11, G12, G22, sc = 1.0;
    if (I.vmode == 0) {
      G00 = G[0]; G01 = G[1]; G02 = G[2]; G11 = G[3]; G12 = G[4]; G22 = G[5];
    } else {
      G00 = G[idx]; G01 = G[q3 + idx]; G02 = G[2 * q3 + idx];
      G11 = G[3 * q3 + idx]; G12 = G[4 * q3 + idx]; G22 = G[5 * q3 + idx];
      sc = 1.0 / (w[a] * w[b] * w[c]);  // the stored metric carries the weights
    }
    F0[idx] = sc * (G00 * g0 + G01 * g1 + G02 * g2);
    F1[idx] = sc * (G01 * g0 + G11 * g1 + G12 * g2);
    F2[idx] = sc * (G02 * g0 + G12 * g1 + G22 * g2);
  }
  __syncthreads();
  const double* vt = ev.vol + ev.voff[e];
  double acc = 0;
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    double dv = 0;
    for (int t = 0; t < q; ++t) {
      dv += Dg[a * q + t] * F0[(c * q + b) * q + t];
      dv += Dg[b * q + t] * F1[(c * q + t) * q + a];
      dv += Dg[c * q + t] * F2[(t * q + b) * q + a];
    }
    const double wdet = vt[3 * idx], idet = vt[3 * idx + 1], gsrc = vt[3 * idx + 2];
    double R = gsrc + dv * idet;
    if (I.mass && L.mcoef) R -= L.mcoef[I.mq + idx] / wdet * U[idx];
    acc += wdet * R * R;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = ev.he2p2[e] * red[0];
}

// eta2(e) = volume part + the parts of the mortars on its faces (face-mortar list)
__global__ void est_sum_kernel(LevelView<double> L, const double* __restrict__ vol, const double* __restrict__ face,
                               double* __restrict__ eta2) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo& I = L.einfo[e];
  double s = vol[e];
  for (int f = 0; f < kFaces; ++f)
    for (int r = 0; r < I.fcnt[f]; ++r) s += face[L.fmlist[I.fstart[f] + r] >> 1];
  eta2[e] = s;
}

}  // namespace

size_t apply_lds_bytes(int NM, int QM, int QMM, size_t scalar, bool compact) {
  const size_t a = Layout(NM, QM, compact, false).bytes(scalar), m = mortar_lds_scalars(NM, QMM) * scalar;
  return a > m ? a : m;
}

template <typename T>
void launch_traces(const LevelView<T>& L, const T* x, hipStream_t s, const int* list, long long count) {
  if (!list) count = L.n_elem;
  if (count == 0) return;
  hipLaunchKernelGGL((trace_kernel<T>), dim3(unsigned(count)), dim3(kThreads), 0, s, L, x, list, count);
}

template <typename T>
void launch_faces(const LevelView<T>& L, hipStream_t s) {
  launch_mortars<T>(L, s);
}


template <typename T>
void launch_apply_bucket(const LevelView<T>& L, int n, int q, const int* elems, long long count, const T* x, T* y,
                         hipStream_t s) {
  if (count == 0) return;
#define HPDG_CASE(NN, QQ) \
  if (n == NN && q == QQ) return launch_fixed<T, NN, QQ>(L, elems, count, x, y, s);
  HPDG_CASE(2, 2) HPDG_CASE(2, 3) HPDG_CASE(3, 3) HPDG_CASE(3, 4) HPDG_CASE(4, 4) HPDG_CASE(4, 5)
  HPDG_CASE(5, 5) HPDG_CASE(5, 6) HPDG_CASE(6, 6) HPDG_CASE(6, 7) HPDG_CASE(7, 7) HPDG_CASE(7, 8)
  HPDG_CASE(8, 8) HPDG_CASE(8, 9)
#undef HPDG_CASE
  const size_t lds = Layout(L.nmax, L.qmax, false, false).bytes(sizeof(T));
  hipLaunchKernelGGL((apply_kernel<T, 0, 0>), dim3(unsigned(count)), dim3(kThreads), lds, s, L, elems, count, x, y,
                     BlockStep<T>{});
}

bool apply_block_fusable(int n, int q) {
  // the compact layout of a fixed-degree kernel, whole waves (the step's block mat-vec)
  return n * n * n <= 2 * kThreads && kThreads % 64 == 0 && n >= 2 && n <= 8 && q >= n && q <= n + 1;
}

template <typename T>
void launch_apply_block_cheb(const LevelView<T>& L, int n, int q, const int* elems, long long count, const T* x,
                             const BlockStep<T>& bs, hipStream_t s) {
  if (count == 0) return;
  if (!apply_block_fusable(n, q)) throw Error(-7, "fused smoother step: degree outside the compact layout");
#define HPDG_CASE(NN, QQ) \
  if (n == NN && q == QQ) return launch_fixed<T, NN, QQ, true>(L, elems, count, x, nullptr, s, bs);
  HPDG_CASE(2, 2) HPDG_CASE(2, 3) HPDG_CASE(3, 3) HPDG_CASE(3, 4) HPDG_CASE(4, 4) HPDG_CASE(4, 5)
  HPDG_CASE(5, 5) HPDG_CASE(5, 6) HPDG_CASE(6, 6) HPDG_CASE(6, 7) HPDG_CASE(7, 7) HPDG_CASE(7, 8)
  HPDG_CASE(8, 8) HPDG_CASE(8, 9)
#undef HPDG_CASE
  throw Error(-7, "fused block step: no kernel for this (n, q)");
}

template void launch_apply_block_cheb<double>(const LevelView<double>&, int, int, const int*, long long,
                                              const double*, const BlockStep<double>&, hipStream_t);
template void launch_apply_block_cheb<float>(const LevelView<float>&, int, int, const int*, long long,
                                             const float*, const BlockStep<float>&, hipStream_t);
template void launch_traces<double>(const LevelView<double>&, const double*, hipStream_t, const int*, long long);
template void launch_traces<float>(const LevelView<float>&, const float*, hipStream_t, const int*, long long);
template void launch_faces<double>(const LevelView<double>&, hipStream_t);
template void launch_faces<float>(const LevelView<float>&, hipStream_t);
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

template void launch_apply_bucket<double>(const LevelView<double>&, int, int, const int*, long long, const double*,
                                          double*, hipStream_t);
template void launch_apply_bucket<float>(const LevelView<float>&, int, int, const int*, long long, const float*,
                                         float*, hipStream_t);

size_t est_lds_bytes(int nmax, int qmax) {
  return sizeof(double) * (size_t(nmax) * nmax * nmax + size_t(nmax) * nmax * qmax + size_t(nmax) * qmax * qmax +
                           4 * size_t(qmax) * qmax * qmax);
}

void launch_estimator(const LevelView<double>& L, const double* x, const EstVolume& ev, const EstFace& ef,
                      long long n_tasks, double* vol, double* eta2, hipStream_t s) {
  if (L.n_elem == 0) return;
  launch_traces<double>(L, x, s);
  hipLaunchKernelGGL(est_volume_kernel, dim3(unsigned(L.n_elem)), dim3(kThreads), est_lds_bytes(L.nmax, L.qmax), s,
                     L, x, ev, vol);
  if (n_tasks > 0) {
    const size_t lds = mortar_lds_scalars(L.nmax, L.qmmax) * sizeof(double);
    hipLaunchKernelGGL((mortar_kernel<double, true>), dim3(unsigned(n_tasks)), dim3(64), lds, s, L, n_tasks, ef);
  }
  hipLaunchKernelGGL(est_sum_kernel, dim3(unsigned((L.n_elem + 255) / 256)), dim3(256), 0, s, L, vol, ef.out, eta2);
}

}  // namespace hpdg
