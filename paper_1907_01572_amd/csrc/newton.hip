// gfx950 kernels of the Newton linearisation (Sec. II.D.1, Eq. newtoncorrectionsystem) for
// -lap u = beta (1 + alpha u)^-7:
//   * nl_eval: u at the volume GL points, the nonlinear source N(u)_psi =
//     sum w det J beta (1 + alpha u)^-7 psi and / or the Jacobian mass coefficient
//     w det J c, c = 7 alpha beta (1 + alpha u)^-8;
//   * inject: the state on the next coarser level (each coarse LGL node takes the value of
//     the polynomial of the finer child that contains it; nodes on the cut belong to the
//     lower child);
//   * diag_mass: the point-Jacobi scaling of A + M(u) (diagonal of the mass form added
//     to the stored diagonal of A).
// One workgroup per element, every intermediate in LDS.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace hpdg {

namespace {

constexpr int kNT = 256;

template <typename T>
__device__ inline const T* mat(const T* tab, const TabView& tv, int kind, int n, int q) {
  return tab + tv.off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q];
}

// out[c][b][a] = sum_{k,j,i} B[c][k] B[b][j] B[a][i] in[k][j][i]   (B: [q][n])
template <typename T>
__device__ void lgl_to_gl(const T* B, int n, int q, const T* in, T* t1, T* t2, T* out) {
  for (int idx = threadIdx.x; idx < n * n * q; idx += blockDim.x) {
    const int a = idx % q, kj = idx / q;
    T s = 0;
    for (int i = 0; i < n; ++i) s += B[a * n + i] * in[kj * n + i];
    t1[idx] = s;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, k = idx / (q * q);
    T s = 0;
    for (int j = 0; j < n; ++j) s += B[b * n + j] * t1[(k * n + j) * q + a];
    t2[idx] = s;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q * q * q; idx += blockDim.x) {
    const int ba = idx % (q * q), c = idx / (q * q);
    T s = 0;
    for (int k = 0; k < n; ++k) s += B[c * n + k] * t2[k * q * q + ba];
    out[idx] = s;
  }
  __syncthreads();
}

// out[k][j][i] = sum_{c,b,a} B[c][k] B[b][j] B[a][i] in[c][b][a]   (transposed passes)
template <typename T>
__device__ void gl_to_lgl(const T* B, int n, int q, const T* in, T* t1, T* t2, T* out) {
  for (int idx = threadIdx.x; idx < n * q * q; idx += blockDim.x) {
    const int ba = idx % (q * q), k = idx / (q * q);
    T s = 0;
    for (int c = 0; c < q; ++c) s += B[c * n + k] * in[c * q * q + ba];
    t2[idx] = s;  // [k][b][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n * q; idx += blockDim.x) {
    const int a = idx % q, j = (idx / q) % n, k = idx / (n * q);
    T s = 0;
    for (int b = 0; b < q; ++b) s += B[b * n + j] * t2[(k * q + b) * q + a];
    t1[idx] = s;  // [k][j][a]
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
    const int i = idx % n, kj = idx / n;
    T s = 0;
    for (int a = 0; a < q; ++a) s += B[a * n + i] * t1[kj * q + a];
    out[idx] = s;
  }
  __syncthreads();
}

// LDS: u / result [NM^3], B [QM NM], t1 [NM^2 QM], t2 [NM QM^2], g [QM^3]
size_t lds_elem(int NM, int QM) {
  const size_t n = NM, q = QM;
  return n * n * n + q * n + n * n * q + n * q * q + q * q * q;
}

// kind 0, 1 (puncture-type): wbeta (1 + alpha u)^-7, mass 7 alpha wbeta (1 + alpha u)^-8;
// kind 2 (constant-density star, Sec. III.B): wbeta u^5, mass -5 wbeta u^4
__global__ void __launch_bounds__(kNT) nl_eval_kernel(LevelView<double> L, int kind, const double* __restrict__ u,
                                                      const double* __restrict__ alpha,
                                                      const double* __restrict__ wbeta, double* N,
                                                      double* mcoef, int* bad) {
  extern __shared__ unsigned char smem_raw[];
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int n = I.n, q = I.q, n3 = n * n * n, q3 = q * q * q;
  double* su = reinterpret_cast<double*>(smem_raw);
  double* B = su + L.nmax * L.nmax * L.nmax;
  double* t1 = B + L.qmax * L.nmax;
  double* t2 = t1 + L.nmax * L.nmax * L.qmax;
  double* g = t2 + L.nmax * L.qmax * L.qmax;
  const double* Bg = mat(L.tab, L.tv, 0, n, q);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) su[i] = u[I.off + i];
  for (int i = threadIdx.x; i < q * n; i += blockDim.x) B[i] = Bg[i];
  __syncthreads();
  lgl_to_gl(B, n, q, su, t1, t2, g);
  for (int idx = threadIdx.x; idx < q3; idx += blockDim.x) {
    const long long k = I.mq + idx;
    if (kind == 2) {
      const double v = g[idx], v2 = v * v, v4 = v2 * v2;
      if (mcoef) mcoef[k] = -5.0 * wbeta[k] * v4;
      g[idx] = wbeta[k] * v4 * v;
      continue;
    }
    const double s = 1.0 + alpha[k] * g[idx];
    if (!(s > 0.0)) bad[0] = 1;
    const double s2 = s * s, s4 = s2 * s2;
    const double inv7 = 1.0 / (s4 * s2 * s);
    if (mcoef) mcoef[k] = 7.0 * alpha[k] * wbeta[k] * inv7 / s;
    g[idx] = wbeta[k] * inv7;
  }
  __syncthreads();
  if (!N) return;
  gl_to_lgl(B, n, q, g, t1, t2, su);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) N[I.off + i] = su[i];
}

template <typename T>
__global__ void __launch_bounds__(kNT) diag_mass_kernel(LevelView<T> L, const T* __restrict__ diagA,
                                                        T* __restrict__ dinv) {
  extern __shared__ unsigned char smem_raw[];
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int n = I.n, q = I.q, n3 = n * n * n, q3 = q * q * q;
  T* out = reinterpret_cast<T*>(smem_raw);
  T* B2 = out + L.nmax * L.nmax * L.nmax;
  T* t1 = B2 + L.qmax * L.nmax;
  T* t2 = t1 + L.nmax * L.nmax * L.qmax;
  T* g = t2 + L.nmax * L.qmax * L.qmax;
  const T* Bg = mat(L.tab, L.tv, 0, n, q);
  // diag(M)_{ijk} = sum_{abc} m_abc B_ai^2 B_bj^2 B_ck^2
  for (int i = threadIdx.x; i < q * n; i += blockDim.x) B2[i] = Bg[i] * Bg[i];
  for (int i = threadIdx.x; i < q3; i += blockDim.x) g[i] = (I.mass && L.mcoef) ? L.mcoef[I.mq + i] : T(0);
  __syncthreads();
  gl_to_lgl(B2, n, q, g, t1, t2, out);
  for (int i = threadIdx.x; i < n3; i += blockDim.x) dinv[I.off + i] = T(1) / (diagA[I.off + i] + out[i]);
}

// one workgroup per coarse element; its finer elements come from the restriction lists
template <typename T>
__global__ void __launch_bounds__(kNT) inject_kernel(TransferView<T> V, const T* __restrict__ uf,
                                                     T* __restrict__ uc) {
  extern __shared__ unsigned char smem_raw[];
  T* sf = reinterpret_cast<T*>(smem_raw);
  const long long K = blockIdx.x;
  if (K >= V.n_coarse) return;
  for (int c = V.cstart[K]; c < V.cstart[K + 1]; ++c) {
    const TransferInfo t = V.tinfo[V.clist[c]];
    const int nf = t.nf, nc = t.nc, nf3 = nf * nf * nf, nc3 = nc * nc * nc;
    __syncthreads();  // sf reuse across children
    for (int i = threadIdx.x; i < nf3; i += blockDim.x) sf[i] = uf[t.foff + i];
    __syncthreads();
    const int h0 = t.bits < 0 ? 0 : 1 + (t.bits & 1);
    const int h1 = t.bits < 0 ? 0 : 1 + ((t.bits >> 1) & 1);
    const int h2 = t.bits < 0 ? 0 : 1 + ((t.bits >> 2) & 1);
    const T* Ex = mat(V.tab, V.tv, 9 + h0, nf, nc);  // [nc][nf]
    const T* Ey = mat(V.tab, V.tv, 9 + h1, nf, nc);
    const T* Ez = mat(V.tab, V.tv, 9 + h2, nf, nc);
    for (int idx = threadIdx.x; idx < nc3; idx += blockDim.x) {
      const int i = idx % nc, j = (idx / nc) % nc, l = idx / (nc * nc);
      // coarse node coordinate <= 0 exactly when 2 index <= nc - 1 (symmetric LGL nodes)
      const bool own = (h0 == 0 || (h0 == 1) == (2 * i <= nc - 1)) &&
                       (h1 == 0 || (h1 == 1) == (2 * j <= nc - 1)) &&
                       (h2 == 0 || (h2 == 1) == (2 * l <= nc - 1));
      if (!own) continue;
      T s = 0;
      for (int cz = 0; cz < nf; ++cz) {
        T sy = 0;
        for (int by = 0; by < nf; ++by) {
          T sx = 0;
          for (int ax = 0; ax < nf; ++ax) sx += Ex[i * nf + ax] * sf[ax + nf * (by + nf * cz)];
          sy += Ey[j * nf + by] * sx;
        }
        s += Ez[l * nf + cz] * sy;
      }
      uc[t.coff + idx] = s;
    }
  }
}

template <typename T>
__global__ void symmetrize_dense_kernel(int n, T* A, int lower_to_upper) {
  const long long total = (long long)n * n;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < total;
       k += (long long)gridDim.x * blockDim.x) {
    const int i = int(k % n), j = int(k / n);  // column-major: A[i + n j]
    if (i <= j) continue;                      // (i, j) strictly lower
    if (lower_to_upper) {
      A[j + (long long)n * i] = A[k];
    } else {
      const T m = T(0.5) * (A[k] + A[j + (long long)n * i]);
      A[k] = m;
      A[j + (long long)n * i] = m;
    }
  }
}

unsigned grid_of(long long n) {
  const long long b = (n + kNT - 1) / kNT;
  return unsigned(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

}  // namespace

void launch_nl_eval(const LevelView<double>& L, int kind, const double* u, const double* alpha, const double* wbeta,
                    double* N, double* mcoef, int* bad, hipStream_t s) {
  if (L.n_elem == 0) return;
  const size_t lds = sizeof(double) * lds_elem(L.nmax, L.qmax);
  hipLaunchKernelGGL(nl_eval_kernel, dim3(unsigned(L.n_elem)), dim3(kNT), lds, s, L, kind, u, alpha, wbeta, N,
                     mcoef, bad);
}

template <typename T>
void launch_diag_mass(const LevelView<T>& L, const T* diagA, T* dinv, hipStream_t s) {
  if (L.n_elem == 0) return;
  const size_t lds = sizeof(T) * lds_elem(L.nmax, L.qmax);
  hipLaunchKernelGGL((diag_mass_kernel<T>), dim3(unsigned(L.n_elem)), dim3(kNT), lds, s, L, diagA, dinv);
}

template <typename T>
void launch_inject(const TransferView<T>& V, const T* uf, T* uc, hipStream_t s) {
  if (V.n_coarse == 0) return;
  const size_t lds = sizeof(T) * size_t(V.nmax) * V.nmax * V.nmax;
  hipLaunchKernelGGL((inject_kernel<T>), dim3(unsigned(V.n_coarse)), dim3(kNT), lds, s, V, uf, uc);
}

template <typename T>
void launch_symmetrize_dense(int n, T* A, int lower_to_upper, hipStream_t s) {
  hipLaunchKernelGGL((symmetrize_dense_kernel<T>), dim3(grid_of((long long)n * n)), dim3(kNT), 0, s, n, A,
                     lower_to_upper);
}

template void launch_diag_mass<double>(const LevelView<double>&, const double*, double*, hipStream_t);
template void launch_diag_mass<float>(const LevelView<float>&, const float*, float*, hipStream_t);
template void launch_inject<double>(const TransferView<double>&, const double*, double*, hipStream_t);
template void launch_symmetrize_dense<double>(int, double*, int, hipStream_t);

}  // namespace hpdg
