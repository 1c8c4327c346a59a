// gfx950 kernels of the hpdg library.
//
// apply: one workgroup per element computes y_e = (A x)_e completely: the volume
// stiffness term by sum factorisation through the GL points (Eq. harald-stiff), and the
// SIPG terms of every mortar on its six faces (Eqs. lh2, temp-E) with both sides' traces
// projected onto the mortar's GL points (Fig. mortar: I_p / I_hp by 1-D matrices).  Each
// mortar is evaluated once from each side; every element writes only its own entries,
// so there are no atomics and the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace hpdg {

namespace {

constexpr int kBS = 256;  // threads of the element kernels

template <typename T>
struct Smem {
  T* su;
  T* sy;
  T* A[4];
  T* tA;
  T* tB;
  T* Bm;   // volume interpolation matrix [q][n]
  T* Dg;   // GL collocation derivative [q][q]
  // face work (aliases the volume buffers A / tA / tB)
  T *Fme, *Nme, *so, *Fo, *No, *T1, *Gme, *Go, *CF, *S, *Yf, *Yn;
};

__device__ inline int vidx(int n, int d, int t0, int t1, int k, int i, int j) {
  int c[3];
  c[d] = k;
  c[t0] = i;
  c[t1] = j;
  return c[0] + n * (c[1] + n * c[2]);
}

struct SideMapD {
  int swap, flipA, flipB, halfA, halfB;
};

__device__ inline SideMapD side_map_d(const MortarInfo& M, int side) {
  SideMapD s{0, 0, 0, 0, 0};
  if (side) {
    s.swap = M.orient & 1;
    s.flipA = (M.orient >> 1) & 1;
    s.flipB = (M.orient >> 2) & 1;
    s.halfA = M.sub < 0 ? 0 : 1 + (M.sub & 1);
    s.halfB = M.sub < 0 ? 0 : 1 + ((M.sub >> 1) & 1);
  }
  return s;
}

template <typename T>
__device__ inline const T* tabm(const LevelView<T>& L, int kind, int n, int q) {
  return L.tab + L.tv.off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q];
}

// trace of a volume array u (n^3) on face f: values F and reference normal derivative N
template <typename T>
__device__ void face_trace(const LevelView<T>& L, const T* u, int n, int f, T* F, T* N) {
  const int d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  const int kf = (f & 1) ? n - 1 : 0;
  const T* df = L.tab + L.tv.dface_off[n] + ((f & 1) ? n : 0);
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;
    F[idx] = u[vidx(n, d, t0, t1, kf, i, j)];
    T s = 0;
    for (int k = 0; k < n; ++k) s += df[k] * u[vidx(n, d, t0, t1, k, i, j)];
    N[idx] = s;
  }
}

// face data of one side (F, N on n x n nodes) -> own-frame grid values at the mortar points:
// G[0] = u, G[1] = du/da, G[2] = du/db, G[3] = du/dn (reference derivatives of that side)
template <typename T>
__device__ void interp_side(const LevelView<T>& L, int n, int q, const SideMapD& m, const T* F,
                            const T* N, T* T1, T* G) {
  const T* Ma = tabm(L, 0 + 2 * m.halfA, n, q);
  const T* Da = tabm(L, 1 + 2 * m.halfA, n, q);
  const T* Mb = tabm(L, 0 + 2 * m.halfB, n, q);
  const T* Db = tabm(L, 1 + 2 * m.halfB, n, q);
  const int nq = n * q, qq = q * q;
  for (int idx = threadIdx.x; idx < nq; idx += blockDim.x) {
    const int x = idx % q, j = idx / q;
    const int ra = m.flipA ? q - 1 - x : x;
    T s0 = 0, s1 = 0, s2 = 0;
    for (int i = 0; i < n; ++i) {
      const T f = F[j * n + i];
      s0 += Ma[ra * n + i] * f;
      s1 += Da[ra * n + i] * f;
      s2 += Ma[ra * n + i] * N[j * n + i];
    }
    T1[idx] = s0;
    T1[nq + idx] = s1;
    T1[2 * nq + idx] = s2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < qq; idx += blockDim.x) {
    const int x = idx % q, y = idx / q;
    const int rb = m.flipB ? q - 1 - y : y;
    T g0 = 0, g1 = 0, g2 = 0, g3 = 0;
    for (int j = 0; j < n; ++j) {
      const T mb = Mb[rb * n + j];
      const T a0 = T1[j * q + x];
      g0 += mb * a0;
      g1 += mb * T1[nq + j * q + x];
      g2 += Db[rb * n + j] * a0;
      g3 += mb * T1[2 * nq + j * q + x];
    }
    G[idx] = g0;
    G[qq + idx] = g1;
    G[2 * qq + idx] = g2;
    G[3 * qq + idx] = g3;
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(kBS) apply_kernel(LevelView<T> L, const T* __restrict__ x,
                                                    T* __restrict__ y) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int n = I.n, q = I.q;
  const int n3 = n * n * n, q3 = q * q * q;
  const int NM = L.nmax, QM = L.qmax, QMM = L.qmmax;

  Smem<T> s;
  T* p = sm;
  s.su = p; p += NM * NM * NM;
  s.sy = p; p += NM * NM * NM;
  s.Bm = p; p += QM * NM;
  s.Dg = p; p += QM * QM;
  T* region = p;
  for (int k = 0; k < 4; ++k) { s.A[k] = p; p += QM * QM * QM; }
  const int tsz = NM * QM * (NM > QM ? NM : QM);
  s.tA = p; p += tsz;
  s.tB = p; p += tsz;
  // face buffers alias the volume region
  p = region;
  s.Fme = p; p += NM * NM;
  s.Nme = p; p += NM * NM;
  s.Fo = p; p += NM * NM;
  s.No = p; p += NM * NM;
  s.Yf = p; p += NM * NM;
  s.Yn = p; p += NM * NM;
  s.so = p; p += NM * NM * NM;
  s.T1 = p; p += 3 * NM * QMM;
  s.S = p; p += 3 * NM * QMM;
  s.Gme = p; p += 4 * QMM * QMM;
  s.Go = p; p += 4 * QMM * QMM;
  s.CF = p; p += 4 * QMM * QMM;

  const T* B = tabm(L, 0, n, q);
  const T* Dgg = L.tab + L.tv.dg_off[q];
  const T* w = L.tab + L.tv.w_off[q];
  for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) s.su[idx] = x[I.off + idx];
  for (int idx = threadIdx.x; idx < q * n; idx += blockDim.x) s.Bm[idx] = B[idx];
  for (int idx = threadIdx.x; idx < q * q; idx += blockDim.x) s.Dg[idx] = Dgg[idx];
  __syncthreads();

  // ---- volume: u -> GL values (three 1-D passes) ----
  for (int idx = threadIdx.x; idx < n * n * q; idx += blockDim.x) {
    const int a = idx % q, kj = idx / q;
    T acc = 0;
    for (int i = 0; i < n; ++i) acc += s.Bm[a * n + i] * s.su[kj * n + i];
    s.tA[idx] = acc;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, k = idx / (q * q);
    T acc = 0;
    for (int j = 0; j < n; ++j) acc += s.Bm[b * n + j] * s.tA[(k * n + j) * q + a];
    s.tB[idx] = acc;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int ba = idx % (q * q), c = idx / (q * q);
    T acc = 0;
    for (int k = 0; k < n; ++k) acc += s.Bm[c * n + k] * s.tB[k * q * q + ba];
    s.A[0][idx] = acc;  // [c][b][a]
  }
  __syncthreads();
  // ---- reference gradient at GL points and the metric contraction ----
  const T* G = L.vgeo + I.vgeo;
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    T g0 = 0, g1 = 0, g2 = 0;
    for (int t = 0; t < q; ++t) {
      g0 += s.Dg[a * q + t] * s.A[0][(c * q + b) * q + t];
      g1 += s.Dg[b * q + t] * s.A[0][(c * q + t) * q + a];
      g2 += s.Dg[c * q + t] * s.A[0][(t * q + b) * q + a];
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
    s.A[1][idx] = G00 * g0 + G01 * g1 + G02 * g2;
    s.A[2][idx] = G01 * g0 + G11 * g1 + G12 * g2;
    s.A[3][idx] = G02 * g0 + G12 * g1 + G22 * g2;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
    T r = 0;
    for (int t = 0; t < q; ++t) {
      r += s.Dg[t * q + a] * s.A[1][(c * q + b) * q + t];
      r += s.Dg[t * q + b] * s.A[2][(c * q + t) * q + a];
      r += s.Dg[t * q + c] * s.A[3][(t * q + b) * q + a];
    }
    if (I.mass) r += G[6 * q3 + idx] * s.A[0][idx];
    s.A[0][idx] = r;
  }
  __syncthreads();
  // ---- back to the LGL test functions (transposed passes) ----
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int ba = idx % (q * q), k = idx / (q * q);
    T acc = 0;
    for (int c = 0; c < q; ++c) acc += s.Bm[c * n + k] * s.A[0][c * q * q + ba];
    s.tB[idx] = acc;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n * q; idx += blockDim.x) {
    const int a = idx % q, j = (idx / q) % n, k = idx / (n * q);
    T acc = 0;
    for (int b = 0; b < q; ++b) acc += s.Bm[b * n + j] * s.tB[(k * q + b) * q + a];
    s.tA[idx] = acc;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) {
    const int i = idx % n, kj = idx / n;
    T acc = 0;
    for (int a = 0; a < q; ++a) acc += s.Bm[a * n + i] * s.tA[kj * q + a];
    s.sy[idx] = acc;
  }
  __syncthreads();

  // ---- faces ----
  for (int f = 0; f < 6; ++f) {
    const int cnt = I.fcnt[f];
    if (cnt == 0) continue;
    const int d = f >> 1, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
    face_trace(L, s.su, n, f, s.Fme, s.Nme);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) { s.Yf[idx] = 0; s.Yn[idx] = 0; }
    __syncthreads();
    for (int c = 0; c < cnt; ++c) {
      const int ent = L.fmlist[I.fstart[f] + c];
      const int side = ent & 1;
      const MortarInfo M = L.minfo[ent >> 1];
      const int qm = M.q, qq = qm * qm;
      const int npts = M.gmode ? qq : 1;
      const T* mg = L.mgeo + M.geo;
      const T* wm = L.tab + L.tv.w_off[qm];
      const SideMapD me = side_map_d(M, side);
      interp_side(L, n, qm, me, s.Fme, s.Nme, s.T1, s.Gme);
      const bool interior = M.ep >= 0;
      SideMapD ot{0, 0, 0, 0, 0};
      int od = 0, ot0 = 0, ot1 = 0;
      if (interior && L.self_only) {
        // neighbour taken as zero: its traces vanish (the element's own diagonal block)
        for (int idx = threadIdx.x; idx < 4 * qq; idx += blockDim.x) s.Go[idx] = 0;
        ot = side_map_d(M, 1 - side);
        od = (side ? M.fm : M.fp) >> 1;
        ot0 = od == 0 ? 1 : 0;
        ot1 = od == 2 ? 1 : 2;
        __syncthreads();
      } else if (interior) {
        const int oe = side ? M.em : M.ep, of = side ? M.fm : M.fp;
        const ElemInfo& O = L.einfo[oe];
        const int no = O.n;
        for (int idx = threadIdx.x; idx < no * no * no; idx += blockDim.x) s.so[idx] = x[O.off + idx];
        __syncthreads();
        face_trace(L, s.so, no, of, s.Fo, s.No);
        __syncthreads();
        ot = side_map_d(M, 1 - side);
        interp_side(L, no, qm, ot, s.Fo, s.No, s.T1, s.Go);
        od = of >> 1;
        ot0 = od == 0 ? 1 : 0;
        ot1 = od == 2 ? 1 : 2;
      }
      for (int idx = threadIdx.x; idx < qq; idx += blockDim.x) {
        const int xg = idx % qm, yg = idx / qm;
        const int cc = me.swap ? yg : xg, dd = me.swap ? xg : yg;
        const int rho = cc + qm * dd, pp = M.gmode ? rho : 0;
        const T wS = M.gmode ? mg[6 * npts + pp] : wm[cc] * wm[dd] * mg[6];
        const T sig = mg[7 * npts + pp];
        const T ma = mg[(3 * side + t0) * npts + pp];
        const T mb = mg[(3 * side + t1) * npts + pp];
        const T mn = mg[(3 * side + d) * npts + pp];
        const T u_me = s.Gme[idx];
        const T g_me = ma * s.Gme[qq + idx] + mb * s.Gme[2 * qq + idx] + mn * s.Gme[3 * qq + idx];
        T A, Bc;
        if (interior) {
          const int os = 1 - side;
          const int xo = ot.swap ? dd : cc, yo = ot.swap ? cc : dd;
          const int oidx = xo + qm * yo;
          const T oa = mg[(3 * os + ot0) * npts + pp];
          const T ob = mg[(3 * os + ot1) * npts + pp];
          const T on = mg[(3 * os + od) * npts + pp];
          const T u_o = s.Go[oidx];
          const T g_o = oa * s.Go[qq + oidx] + ob * s.Go[2 * qq + oidx] + on * s.Go[3 * qq + oidx];
          const T jmp = u_me - u_o;
          A = wS * (sig * jmp - T(0.5) * (g_me - g_o));
          Bc = T(-0.5) * wS * jmp;
        } else {
          A = wS * (sig * u_me - g_me);
          Bc = -wS * u_me;
        }
        s.CF[idx] = A;
        s.CF[qq + idx] = Bc * ma;
        s.CF[2 * qq + idx] = Bc * mb;
        s.CF[3 * qq + idx] = Bc * mn;
      }
      __syncthreads();
      // lift onto the own face nodes (transposed own-side interpolation)
      {
        const T* Ma = tabm(L, 0 + 2 * me.halfA, n, qm);
        const T* Da = tabm(L, 1 + 2 * me.halfA, n, qm);
        const T* Mb = tabm(L, 0 + 2 * me.halfB, n, qm);
        const T* Db = tabm(L, 1 + 2 * me.halfB, n, qm);
        const int nq = n * qm;
        for (int idx = threadIdx.x; idx < nq; idx += blockDim.x) {
          const int i = idx % n, yg = idx / n;
          T s1 = 0, s2 = 0, s3 = 0;
          for (int xg = 0; xg < qm; ++xg) {
            const int ra = me.flipA ? qm - 1 - xg : xg;
            const T ma_ = Ma[ra * n + i];
            const int g = yg * qm + xg;
            s1 += ma_ * s.CF[g] + Da[ra * n + i] * s.CF[qq + g];
            s2 += ma_ * s.CF[2 * qq + g];
            s3 += ma_ * s.CF[3 * qq + g];
          }
          s.S[idx] = s1;          // [y][i]
          s.S[nq + idx] = s2;
          s.S[2 * nq + idx] = s3;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
          const int i = idx % n, j = idx / n;
          T yf = 0, yn = 0;
          for (int yg = 0; yg < qm; ++yg) {
            const int rb = me.flipB ? qm - 1 - yg : yg;
            const T mbv = Mb[rb * n + j];
            yf += mbv * s.S[yg * n + i] + Db[rb * n + j] * s.S[nq + yg * n + i];
            yn += mbv * s.S[2 * nq + yg * n + i];
          }
          s.Yf[idx] += yf;
          s.Yn[idx] += yn;
        }
        __syncthreads();
      }
    }
    // add the face contributions: values on the face layer, normal part along the lines
    const int kf = (f & 1) ? n - 1 : 0;
    const T* df = L.tab + L.tv.dface_off[n] + ((f & 1) ? n : 0);
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
      const int i = idx % n, j = idx / n;
      const T yn = s.Yn[idx];
      for (int k = 0; k < n; ++k) {
        T v = df[k] * yn;
        if (k == kf) v += s.Yf[idx];
        s.sy[vidx(n, d, t0, t1, k, i, j)] += v;
      }
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) y[I.off + idx] = s.sy[idx];
}

// ---- element-block Jacobi -------------------------------------------------------------
template <typename T>
__global__ void set_unit_kernel(LevelView<T> L, int j, T value, T* x) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < L.n_elem;
       e += (long long)gridDim.x * blockDim.x) {
    const ElemInfo& I = L.einfo[e];
    if (j < I.n * I.n * I.n) x[I.off + j] = value;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBS) gather_column_kernel(LevelView<T> L, int j, const T* y,
                                                            const long long* boff, T* B) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  if (j >= N) return;
  // the block is symmetric: column j is stored as row j (contiguous)
  for (int i = threadIdx.x; i < N; i += blockDim.x) B[boff[e] + (long long)j * N + i] = y[I.off + i];
}

template <typename T>
__global__ void __launch_bounds__(kBS) symmetrize_kernel(LevelView<T> L, const long long* boff, T* B) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  T* b = B + boff[e];
  // column-major lower triangle (row >= col) holds the result: b[c * N + r], r >= c
  for (long long idx = threadIdx.x; idx < (long long)N * N; idx += blockDim.x) {
    const int r = int(idx % N), c = int(idx / N);
    if (r < c) b[c * (long long)N + r] = b[r * (long long)N + c];
  }
}

__global__ void __launch_bounds__(kBS) blocks_d2f_kernel(LevelView<double> L, const long long* boff,
                                                         const double* B, float* Bf) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const long long N = (long long)I.n * I.n * I.n;
  for (long long idx = threadIdx.x; idx < N * N; idx += blockDim.x) Bf[boff[e] + idx] = float(B[boff[e] + idx]);
}

// per element: z = Binv r (block_cheb: r = b - Ax first, then the Chebyshev update)
template <typename T, bool CHEB>
__global__ void __launch_bounds__(kBS) block_kernel(LevelView<T> L, const long long* boff, const T* Binv,
                                                    const T* b, const T* Ax, T* p, T* x, T alpha, T beta,
                                                    int first) {
  extern __shared__ unsigned char smem_raw[];
  T* r = reinterpret_cast<T*>(smem_raw);
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    r[i] = (CHEB && Ax) ? b[I.off + i] - Ax[I.off + i] : b[I.off + i];
  __syncthreads();
  const T* B = Binv + boff[e];
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    T z = 0;
    for (int j = 0; j < N; ++j) z += B[(long long)j * N + i] * r[j];  // symmetric: row j, col i
    if (CHEB) {
      const T pn = first ? alpha * z : alpha * z + beta * p[I.off + i];
      p[I.off + i] = pn;
      x[I.off + i] += pn;
    } else {
      x[I.off + i] = z;
    }
  }
}

// ---- transfers (Eqs. psi-interpolation, temp-G) -------------------------------------
template <typename T>
__device__ inline const T* prmat(const TransferView<T>& V, int bits, int axis, int nf, int nc) {
  const int half = bits < 0 ? 0 : 1 + ((bits >> axis) & 1);
  return V.tab + V.tv.off[((6 + half) * (kMaxN + 1) + nc) * (kMaxQ + 1) + nf];
}

template <typename T>
__global__ void __launch_bounds__(kBS) prolong_kernel(TransferView<T> V, const T* __restrict__ uc,
                                                      T* __restrict__ uf) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const long long e = blockIdx.x;
  if (e >= V.n_fine) return;
  const TransferInfo t = V.tinfo[e];
  const int nf = t.nf, nc = t.nc, NM = V.nmax;
  T* a = sm;
  T* b = a + NM * NM * NM;
  const T* P0 = prmat(V, t.bits, 0, nf, nc);
  const T* P1 = prmat(V, t.bits, 1, nf, nc);
  const T* P2 = prmat(V, t.bits, 2, nf, nc);
  for (int idx = threadIdx.x; idx < nc * nc * nc; idx += blockDim.x) a[idx] = uc[t.coff + idx];
  __syncthreads();
  for (int idx = threadIdx.x; idx < nc * nc * nf; idx += blockDim.x) {
    const int x = idx % nf, kj = idx / nf;
    T s = 0;
    for (int i = 0; i < nc; ++i) s += P0[x * nc + i] * a[kj * nc + i];
    b[idx] = s;  // [k][j][x]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nc * nf * nf; idx += blockDim.x) {
    const int x = idx % nf, yv = (idx / nf) % nf, k = idx / (nf * nf);
    T s = 0;
    for (int j = 0; j < nc; ++j) s += P1[yv * nc + j] * b[(k * nc + j) * nf + x];
    a[idx] = s;  // [k][y][x]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nf * nf * nf; idx += blockDim.x) {
    const int yx = idx % (nf * nf), z = idx / (nf * nf);
    T s = 0;
    for (int k = 0; k < nc; ++k) s += P2[z * nc + k] * a[k * nf * nf + yx];
    uf[t.foff + idx] += s;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBS) restrict_kernel(TransferView<T> V, const T* __restrict__ rf,
                                                       T* __restrict__ rc) {
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const long long K = blockIdx.x;
  if (K >= V.n_coarse) return;
  const int NM = V.nmax;
  T* a = sm;
  T* b = a + NM * NM * NM;
  T* acc = b + NM * NM * NM;
  const int c0 = V.cstart[K], c1 = V.cstart[K + 1];
  const int nc = V.tinfo[V.clist[c0]].nc;
  const long long coff = V.tinfo[V.clist[c0]].coff;
  for (int idx = threadIdx.x; idx < nc * nc * nc; idx += blockDim.x) acc[idx] = 0;
  for (int ci = c0; ci < c1; ++ci) {
    const TransferInfo t = V.tinfo[V.clist[ci]];
    const int nf = t.nf;
    const T* P0 = prmat(V, t.bits, 0, nf, nc);
    const T* P1 = prmat(V, t.bits, 1, nf, nc);
    const T* P2 = prmat(V, t.bits, 2, nf, nc);
    __syncthreads();
    for (int idx = threadIdx.x; idx < nf * nf * nf; idx += blockDim.x) a[idx] = rf[t.foff + idx];
    __syncthreads();
    for (int idx = threadIdx.x; idx < nc * nf * nf; idx += blockDim.x) {
      const int yx = idx % (nf * nf), k = idx / (nf * nf);
      T s = 0;
      for (int z = 0; z < nf; ++z) s += P2[z * nc + k] * a[z * nf * nf + yx];
      b[idx] = s;  // [k][y][x]
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nc * nc * nf; idx += blockDim.x) {
      const int x = idx % nf, j = (idx / nf) % nc, k = idx / (nf * nc);
      T s = 0;
      for (int yv = 0; yv < nf; ++yv) s += P1[yv * nc + j] * b[(k * nf + yv) * nf + x];
      a[idx] = s;  // [k][j][x]
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nc * nc * nc; idx += blockDim.x) {
      const int i = idx % nc, kj = idx / nc;
      T s = 0;
      for (int x = 0; x < nf; ++x) s += P0[x * nc + i] * a[kj * nf + x];
      acc[idx] += s;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < nc * nc * nc; idx += blockDim.x) rc[coff + idx] = acc[idx];
}

// ---- vectors -------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(long long n, T v, T* x) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}
template <typename T>
__global__ void copy_kernel(long long n, const T* x, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}
template <typename T>
__global__ void axpby_kernel(long long n, T a, const T* x, T b, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
template <typename T>
__global__ void cheb_kernel(long long n, const T* b, const T* Ax, const T* dinv, T* p, T* x, T alpha,
                            T beta, int first) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    T r = Ax ? b[i] - Ax[i] : b[i];  // Ax == null: x is zero
    if (dinv) r *= dinv[i];
    const T pn = first ? alpha * r : alpha * r + beta * p[i];
    p[i] = pn;
    x[i] += pn;
  }
}
template <typename T>
__global__ void scale_kernel(long long n, const T* a, const T* x, T* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a[i] * x[i];
}
__global__ void d2f_kernel(long long n, const double* x, float* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = float(x[i]);
}
__global__ void f2d_kernel(long long n, const float* x, double* y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = double(x[i]);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block sum in a fixed order (wave shuffles, then wave 0 over the wave sums)
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0;
  if (wv == 0) {
    t = lane < int(blockDim.x >> 6) ? red[lane] : 0.0;
    t = wave_sum(t);
  }
  __syncthreads();
  return t;
}

template <typename T>
__global__ void __launch_bounds__(256) dense_matvec_kernel(int n, const T* A, const T* x, T* y) {
  __shared__ double red[8];
  const int row = blockIdx.x;
  double s = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) s += double(A[(long long)row * n + j]) * double(x[j]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) y[row] = T(s);
}

// partial sums of k dot products; block b writes partials[j * kRedBlocks + b]
__global__ void __launch_bounds__(256) dot_partial_kernel(long long n, const double* a, const double* b,
                                                          double* partials) {
  __shared__ double red[8];
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    s += a[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) dot3_partial_kernel(long long n, const double* v, const double* r,
                                                           const double* w, const double* q,
                                                           double* partials) {
  __shared__ double red[8];
  double s0 = 0, s1 = 0, s2 = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double vi = v[i];
    s0 += vi * r[i];
    s1 += vi * w[i];
    if (q) s2 += vi * q[i];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = s0;
    partials[kRedBlocks + blockIdx.x] = s1;
    partials[2 * kRedBlocks + blockIdx.x] = s2;
  }
}

// out[j] = sum_b partials[j * kRedBlocks + b], j < k
__global__ void __launch_bounds__(256) reduce_final_kernel(const double* partials, int k, double* out) {
  __shared__ double red[8];
  for (int j = 0; j < k; ++j) {
    double s = 0;
    for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x) s += partials[j * kRedBlocks + b];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// FCG scalars in sc: [0] alpha = v.r, [1] beta = v.w, [2] gamma = v.q_{k-1},
// [3] rho_{k-1} -> rho_k, [5] gamma / rho_{k-1}, [6] alpha / rho_k, [7] r.r, [8] breakdown
__global__ void fcg_scalar_kernel(double* sc, int first) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double alpha = sc[0], beta = sc[1], gamma = sc[2];
  double rho, c1;
  if (first) {
    rho = beta;
    c1 = 0.0;
  } else {
    const double rp = sc[3];
    c1 = gamma / rp;
    rho = beta - gamma * c1;
  }
  const bool bad = !(rho > 0.0) || !isfinite(rho) || !isfinite(alpha);
  sc[8] = bad ? 1.0 : sc[8];
  sc[5] = c1;
  sc[6] = bad ? 0.0 : alpha / rho;
  sc[3] = bad ? sc[3] : rho;
}

__global__ void __launch_bounds__(256) fcg_update_kernel(long long n, const double* v, const double* w,
                                                         double* d, double* q, double* u, double* r,
                                                         const double* sc, double* partials, int first) {
  __shared__ double red[8];
  const double c1 = sc[5], step = sc[6];
  double s = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double di = first ? v[i] : v[i] - c1 * d[i];
    const double qi = first ? w[i] : w[i] - c1 * q[i];
    d[i] = di;
    q[i] = qi;
    u[i] += step * di;
    const double ri = r[i] - step * qi;
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

inline int grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return int(g);
}

}  // namespace

size_t apply_lds_bytes(int NM, int QM, int QMM, size_t scalar) {
  const size_t tsz = size_t(NM) * QM * (NM > QM ? NM : QM);
  const size_t vol = 4 * size_t(QM) * QM * QM + 2 * tsz;
  const size_t face = 6 * size_t(NM) * NM + size_t(NM) * NM * NM + 6 * size_t(NM) * QMM +
                      12 * size_t(QMM) * QMM;
  const size_t fixed = 2 * size_t(NM) * NM * NM + size_t(QM) * NM + size_t(QM) * QM;
  return scalar * (fixed + (vol > face ? vol : face));
}

template <typename T>
void launch_apply(const LevelView<T>& L, const T* x, T* y, hipStream_t s) {
  if (L.n_elem == 0) return;
  const size_t lds = apply_lds_bytes(L.nmax, L.qmax, L.qmmax, sizeof(T));
  hipLaunchKernelGGL(apply_kernel<T>, dim3(unsigned(L.n_elem)), dim3(kBS), lds, s, L, x, y);
}

template <typename T>
void launch_set_unit(const LevelView<T>& L, int j, T value, T* x, hipStream_t s) {
  hipLaunchKernelGGL(set_unit_kernel<T>, dim3(grid_for(L.n_elem)), dim3(256), 0, s, L, j, value, x);
}
template <typename T>
void launch_gather_column(const LevelView<T>& L, int j, const T* y, const long long* boff, T* B,
                          hipStream_t s) {
  hipLaunchKernelGGL(gather_column_kernel<T>, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, j, y, boff, B);
}
template <typename T>
void launch_symmetrize_blocks(const LevelView<T>& L, const long long* boff, T* B, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel<T>, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, boff, B);
}
void launch_blocks_d2f(const LevelView<double>& L, const long long* boff, const double* B, float* Bf,
                       hipStream_t s) {
  hipLaunchKernelGGL(blocks_d2f_kernel, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, boff, B, Bf);
}
template <typename T>
void launch_block_apply(const LevelView<T>& L, const long long* boff, const T* Binv, const T* r, T* z,
                        hipStream_t s) {
  const size_t lds = sizeof(T) * size_t(L.nmax) * L.nmax * L.nmax;
  hipLaunchKernelGGL((block_kernel<T, false>), dim3(unsigned(L.n_elem)), dim3(kBS), lds, s, L, boff, Binv,
                     r, (const T*)nullptr, (T*)nullptr, z, T(0), T(0), 0);
}
template <typename T>
void launch_block_cheb(const LevelView<T>& L, const long long* boff, const T* Binv, const T* b,
                       const T* Ax, T* p, T* x, T alpha, T beta, int first, hipStream_t s) {
  const size_t lds = sizeof(T) * size_t(L.nmax) * L.nmax * L.nmax;
  hipLaunchKernelGGL((block_kernel<T, true>), dim3(unsigned(L.n_elem)), dim3(kBS), lds, s, L, boff, Binv,
                     b, Ax, p, x, alpha, beta, first);
}

template <typename T>
void launch_prolong_add(const TransferView<T>& V, const T* uc, T* uf, hipStream_t s) {
  const size_t lds = sizeof(T) * 2 * size_t(V.nmax) * V.nmax * V.nmax;
  hipLaunchKernelGGL(prolong_kernel<T>, dim3(unsigned(V.n_fine)), dim3(kBS), lds, s, V, uc, uf);
}

template <typename T>
void launch_restrict(const TransferView<T>& V, const T* rf, T* rc, hipStream_t s) {
  const size_t lds = sizeof(T) * 3 * size_t(V.nmax) * V.nmax * V.nmax;
  hipLaunchKernelGGL(restrict_kernel<T>, dim3(unsigned(V.n_coarse)), dim3(kBS), lds, s, V, rf, rc);
}

template <typename T>
void launch_fill(long long n, T value, T* x, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, value, x);
}
template <typename T>
void launch_copy(long long n, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
}
template <typename T>
void launch_axpby(long long n, T a, const T* x, T b, T* y, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, b, y);
}
template <typename T>
void launch_cheb_update(long long n, const T* b, const T* Ax, const T* dinv, T* p, T* x, T alpha,
                        T beta, int first, hipStream_t s) {
  hipLaunchKernelGGL(cheb_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, b, Ax, dinv, p, x, alpha,
                     beta, first);
}
template <typename T>
void launch_scale(long long n, const T* a, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, a, x, y);
}
void launch_convert_d2f(long long n, const double* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(d2f_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
}
void launch_convert_f2d(long long n, const float* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(f2d_kernel, dim3(grid_for(n)), dim3(256), 0, s, n, x, y);
}
template <typename T>
void launch_dense_matvec(int n, const T* A, const T* x, T* y, hipStream_t s) {
  hipLaunchKernelGGL(dense_matvec_kernel<T>, dim3(n), dim3(256), 0, s, n, A, x, y);
}
void launch_dot(long long n, const double* a, const double* b, double* partials, double* out,
                hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, n, a, b, partials);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, s, partials, 1, out);
}
void launch_dot3(long long n, const double* v, const double* r, const double* w, const double* q,
                 double* partials, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot3_partial_kernel, dim3(kRedBlocks), dim3(256), 0, s, n, v, r, w, q, partials);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, s, partials, 3, out);
}
void launch_fcg_scalars(double* sc, int first, hipStream_t s) {
  hipLaunchKernelGGL(fcg_scalar_kernel, dim3(1), dim3(64), 0, s, sc, first);
}
void launch_fcg_update(long long n, const double* v, const double* w, double* d, double* q, double* u,
                       double* r, double* sc, double* partials, int first, hipStream_t s) {
  hipLaunchKernelGGL(fcg_update_kernel, dim3(kRedBlocks), dim3(256), 0, s, n, v, w, d, q, u, r, sc,
                     partials, first);
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, s, partials, 1, sc + 7);
}

#define HPDG_INST(T)                                                                            \
  template void launch_apply<T>(const LevelView<T>&, const T*, T*, hipStream_t);                \
  template void launch_prolong_add<T>(const TransferView<T>&, const T*, T*, hipStream_t);       \
  template void launch_restrict<T>(const TransferView<T>&, const T*, T*, hipStream_t);          \
  template void launch_fill<T>(long long, T, T*, hipStream_t);                                  \
  template void launch_copy<T>(long long, const T*, T*, hipStream_t);                           \
  template void launch_axpby<T>(long long, T, const T*, T, T*, hipStream_t);                    \
  template void launch_cheb_update<T>(long long, const T*, const T*, const T*, T*, T*, T, T, int, \
                                      hipStream_t);                                             \
  template void launch_dense_matvec<T>(int, const T*, const T*, T*, hipStream_t);           \
  template void launch_scale<T>(long long, const T*, const T*, T*, hipStream_t);               \
  template void launch_set_unit<T>(const LevelView<T>&, int, T, T*, hipStream_t);              \
  template void launch_gather_column<T>(const LevelView<T>&, int, const T*, const long long*, T*, \
                                        hipStream_t);                                           \
  template void launch_symmetrize_blocks<T>(const LevelView<T>&, const long long*, T*, hipStream_t); \
  template void launch_block_apply<T>(const LevelView<T>&, const long long*, const T*, const T*, T*, \
                                      hipStream_t);                                             \
  template void launch_block_cheb<T>(const LevelView<T>&, const long long*, const T*, const T*,   \
                                     const T*, T*, T*, T, T, int, hipStream_t);
HPDG_INST(double)
HPDG_INST(float)
#undef HPDG_INST

}  // namespace hpdg
