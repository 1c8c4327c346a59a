// Element-centric operator kernel of the hpdg library: y = A x (Eq. lh2 in the nodal basis of
// Eq. Lagrange_Basis) for the elements whose map is affine and axis-aligned, with a constant k
// and no mass term, in one launch per degree.
//
// On such an element the metric of Eq. stiffness-3 is a constant diagonal G = diag(g0, g1, g2)
// (det J, J^-1 J^-T and k folded in), every volume and face integrand is a polynomial that the
// Gauss rules of Eq. harald-stiff integrate exactly, and the integrals factor into the exact 1-D
// mass and stiffness matrices M and K of the LGL basis:
//
//   A_vol = g0 K (x) M (x) M + g1 M (x) K (x) M + g2 M (x) M (x) K      (axes x, y, z)
//
// A face with normal axis d is a constant-coefficient 2-D integral over the other two axes:
// with S the surface Jacobian, sigma the penalty (Eq. penaltyparameter), mn and mo the two
// sides' normal coefficients (k J^-T n along their own normal axes) and h = 1/2 on interior
// faces (1 on Dirichlet faces), the SIPG terms of Eq. temp-E for the test functions of this
// element are the face mass matrix M (x) M applied to
//
//   A = (sigma u - h mn du/dn) - P(sigma u' - h mo du'/dn')    (times the test function)
//   B = -h (u - P u')                                          (times mn dpsi/dn)
//
// at the element's face nodes, where u, du/dn are this side's trace and u', du'/dn' the
// neighbour's (read from its coefficients, through the face orientation), and P is the L2
// projection of the neighbour's face polynomials onto this element's degree (the identity for
// equal degrees, their interpolation when the neighbour's degree is lower); its product with M
// is the exact mixed mass matrix of the two bases, so P realises the p-mortar of Fig. mortar
// exactly.  Writing F_d for the face terms of the faces normal to d spread along the lines in d
// (A at the face layer, mn B l_m'(+-1) at node m of the line), the whole apply is
//
//   y = M_x M_y (g2 K_z u + F_z) + M_y M_z (g0 K_x u + F_x) + M_x M_z (g1 K_y u + F_y)
//
// eight 1-D passes of n x n matrices.  Each element is handled by n^2 threads of one wavefront
// (several elements per wavefront for p <= 2, p = 3), each thread holding one line of the
// element along the current axis in registers; between passes along different axes the lines
// are exchanged through LDS (five exchanges).  The 1-D matrices are uniform across the wavefront
// and are read through scalar loads.  Neighbour coefficients come straight from x (their
// repeated reads are served by the caches), so the apply moves x and y once plus the records; no
// face traces or face slots are written.  Faces that this form does not cover (2:1 faces, faces
// to curved or variable-k elements) are evaluated by the mortar kernel, whose lifted terms
// (face slots) the element adds.  Optionally the kernel ends in the point-Jacobi Chebyshev step
// of Alg. 4 (r = b - A x, z = diag(A)^-1 r, p = alpha z + beta p, x' = x + p), writing x' to a
// second vector so that neighbours still read the old x.
#include <hip/hip_runtime.h>

#include "apply_common.hpp"
#include "device.hpp"

namespace hpdg {

namespace {

constexpr int kMass1 = 12, kStiff1 = 13, kProj = 14;  // OpTable kinds

// out = Mt in along a line (Mt row-major n x n)
template <typename T, int N>
__device__ __forceinline__ void pass(const T* __restrict__ Mt, const T (&in)[N], T (&out)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) acc += Mt[r * N + c] * in[c];
    out[r] = acc;
  }
}

// the neighbour's trace at its face node (ia, ib): value and reference normal derivative
template <typename T, int NN>
__device__ __forceinline__ void neighbour_trace(const T* __restrict__ xo, const T* __restrict__ dfo, int nf, int ia,
                                                int ib, T& u, T& dn) {
  const int d = nf >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  const T* p = xo + vidx(NN, d, t0, t1, 0, ia, ib);
  const int sd = d == 0 ? 1 : (d == 1 ? NN : NN * NN);
  T v[NN];
#pragma unroll
  for (int m = 0; m < NN; ++m) v[m] = p[m * sd];
  u = (nf & 1) ? v[NN - 1] : v[0];
  dn = 0;
#pragma unroll
  for (int m = 0; m < NN; ++m) dn += dfo[m] * v[m];
}

// runtime neighbour degree (mixed-degree levels): nn <= kFastMaxN
template <typename T>
__device__ __forceinline__ void neighbour_trace_rt(const T* __restrict__ xo, const T* __restrict__ dfo, int nn,
                                                   int nf, int ia, int ib, T& u, T& dn) {
  const int d = nf >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  const T* p = xo + vidx(nn, d, t0, t1, 0, ia, ib);
  const int sd = d == 0 ? 1 : (d == 1 ? nn : nn * nn);
  u = p[((nf & 1) ? nn - 1 : 0) * sd];
  dn = 0;
#pragma unroll
  for (int m = 0; m < kFastMaxN; ++m)
    if (m < nn) dn += dfo[m] * p[m * sd];
}

// node (a, b) of this side's face -> the neighbour's face coordinates (n nodes per axis)
__device__ __forceinline__ void map_node(int map, int n, int a, int b, int& ia, int& ib) {
  ia = (map & 1) ? b : a;
  ib = (map & 1) ? a : b;
  if (map & 2) ia = n - 1 - ia;
  if (map & 4) ib = n - 1 - ib;
}

// The neighbour side of face f at this thread's face node, for neighbours of this element's
// degree: returns q1 = -S P(sigma u' - mo/2 du'/dn') and q2 = S mn h P u' (P the identity), the
// parts of S A and S B that the neighbour contributes (0 on boundary faces and with self_only).
template <typename T, int N>
__device__ __forceinline__ void neighbour_part(const LevelView<T>& L, const T* __restrict__ tab, const T* __restrict__ x,
                                               const FaceLink& fl, int a, int b, T& q1, T& q2) {
  q1 = 0;
  q2 = 0;
  const int meta = fl.meta;
  if ((meta & 3) != 1 || L.self_only || ((meta >> 2) & 31) != N) return;
  const int nf = (meta >> 7) & 7, map = (meta >> 10) & 7;
  int ia, ib;
  map_node(map, N, a, b, ia, ib);
  T uo, dno;
  neighbour_trace<T, N>(x + fl.nb, tab + L.tv.dface_off[N] + (nf & 1) * N, nf, ia, ib, uo, dno);
  const T* cf = L.fcoef + 4 * fl.coef;
  const T S = cf[0], sig = cf[1], mn = cf[2], mo = cf[3];
  q1 = -S * (sig * uo - T(0.5) * mo * dno);
  q2 = T(0.5) * S * mn * uo;
}

// Neighbours of another degree nn on the two faces normal to axis d (mixed-degree groups): their
// face data at their nn^2 nodes in this side's axes, then the projection P (N x nn) along b and
// along a, into q1, q2 (as neighbour_part).  A neighbour of higher degree is read from the face
// trace it wrote (2 scalars per node), one of lower degree from its coefficients (one node per
// thread).  Every thread of the workgroup calls this; it synchronises twice.
template <typename T, int N>
__device__ __forceinline__ void mixed_parts(const LevelView<T>& L, const T* __restrict__ tab, const T* __restrict__ x,
                                            const FaceLink* fl, int a, int b, bool act, T* scr, int nx, T* q1, T* q2) {
  constexpr int N2 = N * N;
  const int lt = a + N * b;
  const int psz = 2 * nx * nx + 2 * nx * N;
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int meta = fl[fi].meta, nn = (meta >> 2) & 31;
    if (act && (meta & 3) == 1 && !L.self_only && nn != N) {
      const int nf = (meta >> 7) & 7, map = (meta >> 10) & 7;
      const T* cf = L.fcoef + 4 * fl[fi].coef;
      const T sig = cf[1], mo = cf[3];
      T* Ga = scr + fi * psz;
      T* Gb = Ga + nx * nx;
      if (nn > N) {
        const T* __restrict__ nt = L.trace + fl[fi].nb;
#pragma unroll 4
        for (int g = lt; g < nn * nn; g += N2) {
          const int ga = g % nn, gb = g / nn;
          int ia, ib;
          map_node(map, nn, ga, gb, ia, ib);
          const T uo = nt[ia + nn * ib], dno = nt[nn * nn + ia + nn * ib];
          Ga[g] = sig * uo - T(0.5) * mo * dno;
          Gb[g] = uo;
        }
      } else if (lt < nn * nn) {
        const int ga = lt % nn, gb = lt / nn;
        int ia, ib;
        map_node(map, nn, ga, gb, ia, ib);
        const int d = nf >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        const T* p = x + fl[fi].nb + vidx(nn, d, t0, t1, 0, ia, ib);
        const int sd = d == 0 ? 1 : (d == 1 ? nn : nn * nn);
        const T* dfo = tab + L.tv.dface_off[nn] + (nf & 1) * nn;
        const T uo = p[((nf & 1) ? nn - 1 : 0) * sd];
        T dno = 0;
#pragma unroll 4
        for (int m = 0; m < nn; ++m) dno += dfo[m] * p[m * sd];
        Ga[lt] = sig * uo - T(0.5) * mo * dno;
        Gb[lt] = uo;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int meta = fl[fi].meta, nn = (meta >> 2) & 31;
    if (act && (meta & 3) == 1 && !L.self_only && nn != N) {
      const T* P = tab + L.tv.off[(kProj * (kMaxN + 1) + nn) * (kMaxQ + 1) + N];  // [N][nn]
      const T* Ga = scr + fi * psz;
      const T* Gb = Ga + nx * nx;
      T* Ta = scr + fi * psz + 2 * nx * nx;
      T* Tb = Ta + nx * N;
      for (int g = lt; g < nn * N; g += N2) {  // T[ga][j] = sum_gb P[j][gb] G[ga][gb]
        const int ga = g % nn, j = g / nn;
        T sa = 0, sb = 0;
#pragma unroll 4
        for (int gb = 0; gb < nn; ++gb) {
          const T pv = P[j * nn + gb];
          sa += pv * Ga[ga + nn * gb];
          sb += pv * Gb[ga + nn * gb];
        }
        Ta[g] = sa;
        Tb[g] = sb;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int meta = fl[fi].meta, nn = (meta >> 2) & 31;
    if (act && (meta & 3) == 1 && !L.self_only && nn != N) {
      const T* P = tab + L.tv.off[(kProj * (kMaxN + 1) + nn) * (kMaxQ + 1) + N];
      const T* Ta = scr + fi * psz + 2 * nx * nx;
      const T* Tb = Ta + nx * N;
      T sa = 0, sb = 0;
#pragma unroll 4
      for (int ga = 0; ga < nn; ++ga) {
        const T pv = P[a * nn + ga];
        sa += pv * Ta[ga + nn * b];
        sb += pv * Tb[ga + nn * b];
      }
      const T* cf = L.fcoef + 4 * fl[fi].coef;
      q1[fi] = -cf[0] * sa;
      q2[fi] = T(0.5) * cf[0] * cf[2] * sb;
    }
  }
}

// Face terms of the two faces normal to axis d, added to F (the thread's line along d, nodes
// m = 0..N-1) from the thread's line u of the element; the thread holds face node (a, b) of
// both faces; q1, q2: the neighbour parts (neighbour_part, mixed_parts).
template <typename T, int N>
__device__ __forceinline__ void faces_along(const LevelView<T>& L, const T* __restrict__ tab, const T* __restrict__ x,
                                            const T* __restrict__ df, const FaceLink* fl, const T* q1m,
                                            const T* q2m, int a, int b, bool act, const T (&u)[N], T (&F)[N]) {
  if (!act) return;
#pragma unroll
  for (int fi = 0; fi < 2; ++fi) {
    const int kind = fl[fi].meta & 3;
    if (kind != 1 && kind != 2) continue;
    // the neighbour's part: same degree read here, another degree from mixed_parts
    T q1, q2;
    neighbour_part<T, N>(L, tab, x, fl[fi], a, b, q1, q2);
    if (q1m) {
      q1 += q1m[fi];
      q2 += q2m[fi];
    }
    const T* cf = L.fcoef + 4 * fl[fi].coef;
    const T S = cf[0], sig = cf[1], mn = cf[2];
    const T* dfs = df + fi * N;
    const int layer = fi ? N - 1 : 0;
    const T us = u[layer];
    T dns = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) dns += dfs[m] * u[m];
    const T h = kind == 1 ? T(0.5) : T(1);
    const T Smn = S * mn;
    const T A = S * sig * us - h * Smn * dns + q1;
    const T B = -h * Smn * us + q2;
    F[layer] += A;
#pragma unroll
    for (int m = 0; m < N; ++m) F[m] += dfs[m] * B;
  }
}

// LDS layout of an element's exchange buffers: node (i, j, k) at i + P1 j + P2 k, three buffers
// of P2 n scalars, elements ES scalars apart.  The strides are chosen (by a search over small
// paddings) so that the three exchange patterns (lines along z, x and y spread over the lanes)
// meet few bank conflicts in groups of 16 lanes of 8 bytes: the unpadded layout puts a line
// along x at a stride of n scalars, a 16-way conflict for n = 8.
struct Pad {
  int p1, p2, es;
};
template <int N>
constexpr Pad fast_pad() {
  return N == 2 ? Pad{2, 5, 36}
       : N == 3 ? Pad{3, 9, 91}
       : N == 4 ? Pad{4, 19, 228}
       : N == 5 ? Pad{5, 25, 377}
       : N == 6 ? Pad{6, 36, 648}
       : N == 7 ? Pad{7, 49, 1029}
                : Pad{9, 72, 1728};
}
// projection scratch of a mixed-degree group (two faces at the largest neighbour degree), and
// whether it fits in the exchange buffers (free while the projections run, before the volume
// passes); otherwise it follows them
template <int N>
constexpr int fast_scr_scalars() {
  constexpr int nx = kFastMaxN + 1;
  return 2 * (2 * nx * nx + 2 * nx * N);
}
template <int N>
constexpr bool fast_scr_shared() { return fast_scr_scalars<N>() <= 3 * fast_pad<N>().p2 * N; }
// scalars per element: the exchange buffers and a separate projection scratch when needed (kept a
// multiple of 16 scalars so the element stride keeps its bank offset)
template <int N, bool MIX>
constexpr int fast_elem_scalars() {
  constexpr int scr = MIX && !fast_scr_shared<N>() ? fast_scr_scalars<N>() : 0;
  return fast_pad<N>().es + (scr + 15) / 16 * 16;
}

// at least this many waves per SIMD: the register budget of each instantiation (uniform-degree
// groups: 128 VGPRs, 168 for the fused step from p = 6 up; mixed-degree groups, which hold the
// projection stage's results: 168, and 256 from p = 5 up)
template <int N, bool MIX, bool FUSE>
constexpr int fast_waves() { return MIX ? (N >= 6 ? 2 : 3) : (FUSE && N >= 7 ? 3 : 4); }

template <typename T, int N, bool MIX, bool FUSE>
__global__ void __launch_bounds__(64, (fast_waves<N, MIX, FUSE>())) fast_kernel(LevelView<T> L, FastBucket<T> fb, const T* __restrict__ x,
                                                  T* __restrict__ y, FastStep<T> st) {
  constexpr int N2 = N * N;
  constexpr int EPW = N2 <= 64 ? 64 / N2 : 1;
  extern __shared__ unsigned char smem_raw[];
  T* smem = reinterpret_cast<T*>(smem_raw);
  const T* __restrict__ tab = L.tab;
  const int nx = fb.nx;
  const int t = threadIdx.x;
  const int es = t / N2, lt = t - es * N2;
  const int li = lt % N, lj = lt / N;
  const long long loc = (long long)xcd_remap(blockIdx.x, gridDim.x) * EPW + es;
  const bool act = es < EPW && loc < fb.count;
  const long long gi = fb.start + (act ? loc : 0);
  constexpr Pad PD = fast_pad<N>();
  constexpr int P1 = PD.p1, P2 = PD.p2, BS = P2 * N;
  T* B0 = smem + (act ? es : 0) * fast_elem_scalars<N, MIX>();
  T* B1 = B0 + BS;
  T* B2 = B1 + BS;
  T* scr = fast_scr_shared<N>() ? B0 : B2 + BS;
  const int zi = li + P1 * lj;  // z line of thread (i, j): zi + P2 k
  const int xi = P1 * li + P2 * lj;  // x line of thread (j, k): xi + i
  const int yi = li + P2 * lj;  // y line of thread (i, k): yi + P1 j
  const T* __restrict__ M1 = fb.M1;
  const T* __restrict__ K1 = fb.K1;
  const T* __restrict__ df = fb.df;
  // records of this element (bucket order): dof offset, diagonal metric, six face records; then
  // its coefficients and the neighbour parts of its same-degree faces, all loads issued up front
  const long long off = act ? L.fe_off[gi] : 0;
  T g0 = 0, g1 = 0, g2 = 0;
  FaceLink fl[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) fl[f] = FaceLink{0, 0, 0};
  if (act) {
    g0 = L.fe_g[3 * gi];
    g1 = L.fe_g[3 * gi + 1];
    g2 = L.fe_g[3 * gi + 2];
#pragma unroll
    for (int f = 0; f < 6; ++f) fl[f] = L.flink[6 * gi + f];
  }
  T q1[6], q2[6];  // mixed-degree groups: the parts of neighbours of another degree
#pragma unroll
  for (int f = 0; f < 6; ++f) q1[f] = q2[f] = 0;
  if constexpr (MIX) {
    // neighbours of another degree, all six faces before the volume passes (the face node of a
    // thread is (li, lj) on every face)
#pragma unroll
    for (int d = 0; d < 3; ++d) mixed_parts<T, N>(L, tab, x, fl + 2 * d, li, lj, act, scr, nx, q1 + 2 * d, q2 + 2 * d);
    __syncthreads();  // the scratch may be the exchange buffers
  }

  // ---- z: lines along z (thread (i, j)) ----
  T u[N], c[N];
#pragma unroll
  for (int k = 0; k < N; ++k) u[k] = act ? x[off + lt + N2 * k] : T(0);
  pass<T, N>(K1, u, c);
#pragma unroll
  for (int k = 0; k < N; ++k) c[k] *= g2;
  faces_along<T, N>(L, tab, x, df, fl + 4, MIX ? q1 + 4 : nullptr, q2 + 4, li, lj, act, u, c);
  if (act) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      B0[zi + P2 * k] = u[k];
      B1[zi + P2 * k] = c[k];
    }
  }
  __syncthreads();
  // ---- x: lines along x (thread (j, k)) ----
  T w1[N], v1[N];
  {
    T ux[N], cx[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ux[i] = act ? B0[xi + i] : T(0);
      cx[i] = act ? B1[xi + i] : T(0);
    }
    pass<T, N>(K1, ux, w1);
#pragma unroll
    for (int i = 0; i < N; ++i) w1[i] *= g0;
    faces_along<T, N>(L, tab, x, df, fl, MIX ? q1 : nullptr, q2, li, lj, act, ux, w1);
    pass<T, N>(M1, cx, v1);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      B1[xi + i] = w1[i];
      B2[xi + i] = v1[i];
    }
  }
  __syncthreads();
  // ---- y: lines along y (thread (i, k)) ----
  T ya[N], t2[N], w2[N];
  {
    T uy[N], w1y[N], v1y[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int idx = yi + P1 * j;
      uy[j] = act ? B0[idx] : T(0);
      w1y[j] = act ? B1[idx] : T(0);
      v1y[j] = act ? B2[idx] : T(0);
    }
    pass<T, N>(M1, v1y, ya);
    pass<T, N>(M1, w1y, t2);
    pass<T, N>(K1, uy, w2);
#pragma unroll
    for (int j = 0; j < N; ++j) w2[j] *= g1;
    faces_along<T, N>(L, tab, x, df, fl + 2, MIX ? q1 + 2 : nullptr, q2 + 2, li, lj, act, uy, w2);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int j = 0; j < N; ++j) B0[yi + P1 * j] = w2[j];
  }
  __syncthreads();
  // ---- x: M_x of the y-face term ----
  T t3[N];
  {
    T w2x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) w2x[i] = act ? B0[xi + i] : T(0);
    pass<T, N>(M1, w2x, t3);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
      B0[xi + m] = t3[m];
      B1[yi + P1 * m] = t2[m];
      B2[yi + P1 * m] = ya[m];
    }
  }
  __syncthreads();
  if (!act) return;
  // ---- z: y = y_a + M_z (t2 + t3), then the face slots of faces left to the mortar kernel ----
  T acc[N];
  {
    T sm[N];
#pragma unroll
    for (int k = 0; k < N; ++k) sm[k] = B1[zi + P2 * k] + B0[zi + P2 * k];
    pass<T, N>(M1, sm, acc);
#pragma unroll
    for (int k = 0; k < N; ++k) acc[k] += B2[zi + P2 * k];
  }
  bool slots = false;
#pragma unroll
  for (int f = 0; f < 6; ++f) slots = slots || (fl[f].meta & 3) == 3;
  if (slots) {
    const ElemInfo* I = L.einfo + L.fe_id[gi];
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
      if ((L.flink[6 * gi + f].meta & 3) != 3) continue;
      const int cnt = I->fcnt[f];
      const T* sl = L.slot + I->soff + 2LL * (I->fstart[f] - I->fstart[0]) * N2;
      const int d = f >> 1, layer = (f & 1) ? N - 1 : 0;
      const T* dfs = df + (f & 1) * N;
      for (int r = 0; r < cnt; ++r, sl += 2 * N2) {
        if (d == 2) {
          const T vv = sl[lt], nv = sl[N2 + lt];
          acc[layer] += vv;
#pragma unroll
          for (int k = 0; k < N; ++k) acc[k] += dfs[k] * nv;
        } else {
          const int own = d == 0 ? li : lj, oth = d == 0 ? lj : li;
          const T dv = dfs[own];
#pragma unroll
          for (int k = 0; k < N; ++k) {
            const int fidx = oth + N * k;
            acc[k] += dv * sl[N2 + fidx] + (own == layer ? sl[fidx] : T(0));
          }
        }
      }
    }
  }
  if constexpr (FUSE) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const long long idx = off + lt + N2 * k;
      const T z = st.dinv[idx] * (st.b[idx] - acc[k]);
      const T pn = st.first ? st.alpha * z : st.alpha * z + st.beta * st.p[idx];
      st.p[idx] = pn;
      st.xo[idx] = u[k] + pn;
    }
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) y[off + lt + N2 * k] = acc[k];
  }
  if constexpr (MIX) {
    // this element's face traces for its neighbours of lower degree (read by their groups,
    // launched after this one): the value and the normal derivative at face node (li, lj) of x
    // (written last: stores among the volume passes cost registers)
    T* const trb = L.trace + L.fe_toff[gi];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (!(fl[f].meta & (1 << 13))) continue;
      const int d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      const T* p = x + off + vidx(N, d, t0, t1, 0, li, lj);
      const int sd = d == 0 ? 1 : (d == 1 ? N : N2);
      const T* dfs = df + (f & 1) * N;
      T dn = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) dn += dfs[m] * p[m * sd];
      trb[2 * f * N2 + lt] = p[((f & 1) ? N - 1 : 0) * sd];
      trb[(2 * f + 1) * N2 + lt] = dn;
    }
  }
}

template <typename T, int N, bool MIX, bool FUSE>
void launch_n(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, T* y, const FastStep<T>& st,
              hipStream_t s) {
  constexpr int N2 = N * N;
  constexpr int EPW = N2 <= 64 ? 64 / N2 : 1;
  const size_t lds = size_t(EPW) * size_t(fast_elem_scalars<N, MIX>()) * sizeof(T);
  const long long groups = (fb.count + EPW - 1) / EPW;
  hipLaunchKernelGGL((fast_kernel<T, N, MIX, FUSE>), dim3(unsigned(groups)), dim3(64), lds, s, L, fb, x, y, st);
}

template <typename T, bool FUSE>
void launch_fast_impl(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, T* y, const FastStep<T>& st,
                      hipStream_t s) {
  if (fb.count == 0) return;
  const int n = fb.n, nx = fb.nx;
  if (n < 2 || n > kFastMaxN || nx < n || nx > kFastMaxN + 1)
    throw Error(-7, "element-centric apply: degree outside its range");
  const bool mix = nx != n;  // some neighbour of another degree (nx bounds their n)
#define HPDG_FAST(NN)                                         \
  if (n == NN) {                                              \
    if (mix)                                                  \
      launch_n<T, NN, true, FUSE>(L, fb, x, y, st, s);        \
    else                                                      \
      launch_n<T, NN, false, FUSE>(L, fb, x, y, st, s);       \
    return;                                                   \
  }
  HPDG_FAST(2) HPDG_FAST(3) HPDG_FAST(4) HPDG_FAST(5) HPDG_FAST(6) HPDG_FAST(7) HPDG_FAST(8)
#undef HPDG_FAST
}

}  // namespace

template <typename T>
void launch_fast_apply(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, T* y, hipStream_t s) {
  launch_fast_impl<T, false>(L, fb, x, y, FastStep<T>{}, s);
}

template <typename T>
void launch_fast_cheb(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, const FastStep<T>& st,
                      hipStream_t s) {
  launch_fast_impl<T, true>(L, fb, x, nullptr, st, s);
}

template void launch_fast_apply<double>(const LevelView<double>&, const FastBucket<double>&, const double*, double*,
                                        hipStream_t);
template void launch_fast_apply<float>(const LevelView<float>&, const FastBucket<float>&, const float*, float*,
                                       hipStream_t);
template void launch_fast_cheb<double>(const LevelView<double>&, const FastBucket<double>&, const double*,
                                       const FastStep<double>&, hipStream_t);
template void launch_fast_cheb<float>(const LevelView<float>&, const FastBucket<float>&, const float*,
                                      const FastStep<float>&, hipStream_t);

}  // namespace hpdg
