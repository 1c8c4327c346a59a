// gfx950 kernels of the hpdg library besides the operator apply (apply.hip): element-block
// Jacobi, multigrid transfers, Chebyshev / Krylov vector updates, deterministic reductions
// and the dense coarse solve.
#include <hip/hip_runtime.h>

#include "blocks.hpp"
#include "device.hpp"

namespace hpdg {

namespace {

constexpr int kBS = 256;  // threads of the element kernels

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

// consistency of freshly gathered element blocks before their factorisation: the diagonal must
// equal the level's stored diagonal (computed independently on the host) and the block must be
// symmetric; bad[e] = 1 + first offending column of element e, or 0
__global__ void __launch_bounds__(kBS) check_blocks_kernel(LevelView<double> L, const long long* boff,
                                                           const double* B, const double* dinv, int* bad) {
  __shared__ int first;
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  const double* Be = B + boff[e];
  if (threadIdx.x == 0) first = N;
  __syncthreads();
  for (int idx = threadIdx.x; idx < N * N; idx += blockDim.x) {
    const int i = idx % N, j = idx / N;
    const double a = Be[(long long)j * N + i], b = Be[(long long)i * N + j];
    const double dref = 1.0 / dinv[I.off + j];
    const double scale = fabs(Be[(long long)j * N + j]) + fabs(Be[(long long)i * N + i]);
    bool ok = fabs(a - b) <= 1e-9 * scale;
    if (i == j) ok = ok && fabs(a - dref) <= 1e-9 * fabs(dref);
    if (!ok) atomicMin(&first, j);
  }
  __syncthreads();
  if (threadIdx.x == 0) bad[e] = first < N ? first + 1 : 0;
}

// ---- packed symmetric inverse blocks ----------------------------------------------------
// Only the lower triangle of each inverse block is stored (N (N + 1) / 2 scalars for N = n^3),
// in panels of 64 rows: panel rows r0 = 64 P .. r0 + m - 1 (m = min(64, N - r0)) start at
// r0 (r0 + 1) / 2 and hold first the r0 full columns of these rows (column c: m scalars in row
// order), then the panel's diagonal tile column by column (tile column j: rows j .. m - 1).
// A wave reading one column of a panel reads consecutive addresses.
__device__ inline long long packed_index(int N, int r, int c) {  // r >= c
  const int r0 = r & ~63, m = min(64, N - r0), l = r - r0;
  const long long base = (long long)r0 * (r0 + 1) / 2;
  if (c < r0) return base + (long long)c * m + l;
  const int j = c - r0;
  return base + (long long)r0 * m + (long long)j * m - (long long)j * (j - 1) / 2 + (l - j);
}

// bf16: round to nearest even on the upper 16 bits of the FP32 value
__device__ inline uint16_t f2bf(float v) {
  const uint32_t u = __float_as_uint(v);
  return uint16_t((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

template <typename S>
__device__ inline S to_storage(double v) { return S(v); }
template <typename T, typename S>
__device__ inline T from_storage(S v) { return T(v); }

// pack the FP64 inverse blocks (column-major, lower triangle valid: B[c N + r], r >= c)
template <typename S>
__global__ void __launch_bounds__(kBS) pack_blocks_kernel(LevelView<double> L, const long long* boff,
                                                          const double* B, const long long* poff, S* P) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  const double* Be = B + boff[e];
  S* Pe = P + poff[e];
  for (long long idx = threadIdx.x; idx < (long long)N * N; idx += blockDim.x) {
    const int r = int(idx % N), c = int(idx / N);
    if (r >= c) Pe[packed_index(N, r, c)] = to_storage<S>(Be[idx]);
  }
}

// bf16 copies of the symmetric inverse blocks, full (column-major, both triangles): the FP32
// V-cycle's bf16 mode reads these with the row-per-thread kernel below
__global__ void __launch_bounds__(kBS) blocks_bf16_full_kernel(LevelView<double> L, const long long* boff,
                                                               const double* B, uint16_t* Bh) {
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  const double* Be = B + boff[e];
  for (long long idx = threadIdx.x; idx < (long long)N * N; idx += blockDim.x) {
    const int r = int(idx % N), c = int(idx / N);
    const double v = r >= c ? Be[idx] : Be[(long long)r * N + c];  // lower triangle valid
    Bh[boff[e] + idx] = f2bf(float(v));
  }
}

// Chebyshev step with the full bf16 blocks: one thread per row, operands widened to FP32, FP32
// accumulation (the blocks are symmetric, so row i is read as column i: coalesced over i)
__global__ void __launch_bounds__(kBS) block_cheb_bf16_kernel(LevelView<float> L, const long long* boff,
                                                              const uint16_t* Binv, const float* b, const float* Ax,
                                                              float* p, float* x, float alpha, float beta,
                                                              int first) {
  extern __shared__ unsigned char smem_raw[];
  float* r = reinterpret_cast<float*>(smem_raw);
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  for (int i = threadIdx.x; i < N; i += blockDim.x) r[i] = Ax ? b[I.off + i] - Ax[I.off + i] : b[I.off + i];
  __syncthreads();
  const uint16_t* B = Binv + boff[e];
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    float z = 0;
#pragma unroll 8
    for (int j = 0; j < N; ++j) z += bf2f(B[(long long)j * N + i]) * r[j];
    const float pn = first ? alpha * z : alpha * z + beta * p[I.off + i];
    p[I.off + i] = pn;
    x[I.off + i] += pn;
  }
}

// per element, blockDim.x / 64 waves (column block k taken by wave k % waves): z = Binv r with
// Binv symmetric and packed (each stored off-diagonal entry is used twice: for its row and,
// via the wave column sums, for its column); CHEB: r = b - Ax (Ax null: r = b),
// p = alpha z + beta p (first: alpha z), x += p; else x = z. S is the storage type (double or
// float), T the arithmetic type. LDS: r (broadcast reads), then per wave the accumulators of z
// (index i only touched by lane i % 64 of that wave), summed over the waves in a fixed order.
template <typename S, typename T, bool CHEB>
__global__ void __launch_bounds__(512) block_sym_kernel(LevelView<T> L, const long long* poff, const S* P,
                                                        const T* b, const T* Ax, T* p, T* x, T alpha, T beta,
                                                        int first) {
  extern __shared__ unsigned char smem_raw[];
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const int N = I.n * I.n * I.n;
  // the wave index is uniform over the wave: taken into a scalar register, so that the loop
  // control and the block addresses stay scalar
  const int waves = int(blockDim.x >> 6), lane = int(threadIdx.x & 63);
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  T* rs = reinterpret_cast<T*>(smem_raw);
  T* zs = rs + N + wv * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    rs[i] = (CHEB && Ax) ? b[I.off + i] - Ax[I.off + i] : b[I.off + i];
  for (int i = lane; i < N; i += 64) zs[i] = 0;
  __syncthreads();
  packed_block_partial<S, T>(P + poff[e], N, rs, zs, waves, wv, lane);
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    T z = 0;
    for (int w = 0; w < waves; ++w) z += rs[N + w * N + i];
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
                            T beta, int first, T* xo) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    T r = Ax ? b[i] - Ax[i] : b[i];  // Ax == null: x is zero
    if (dinv) r *= dinv[i];
    const T pn = first ? alpha * r : alpha * r + beta * p[i];
    p[i] = pn;
    xo[i] = x[i] + pn;
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

template <typename T>
void launch_set_unit(const LevelView<T>& L, int j, T value, T* x, hipStream_t s) {
  hipLaunchKernelGGL(set_unit_kernel<T>, dim3(grid_for(L.n_elem)), dim3(256), 0, s, L, j, value, x);
}
template <typename T>
void launch_gather_column(const LevelView<T>& L, int j, const T* y, const long long* boff, T* B,
                          hipStream_t s) {
  hipLaunchKernelGGL(gather_column_kernel<T>, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, j, y, boff, B);
}
template <typename S>
void launch_pack_blocks(const LevelView<double>& L, const long long* boff, const double* B, const long long* poff,
                        S* P, hipStream_t s) {
  hipLaunchKernelGGL(pack_blocks_kernel<S>, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, boff, B, poff, P);
}
template void launch_pack_blocks<double>(const LevelView<double>&, const long long*, const double*,
                                         const long long*, double*, hipStream_t);
template void launch_pack_blocks<float>(const LevelView<double>&, const long long*, const double*,
                                        const long long*, float*, hipStream_t);
void launch_blocks_bf16_full(const LevelView<double>& L, const long long* boff, const double* B, uint16_t* Bh,
                             hipStream_t s) {
  hipLaunchKernelGGL(blocks_bf16_full_kernel, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, boff, B, Bh);
}
void launch_block_cheb_bf16(const LevelView<float>& L, const long long* boff, const uint16_t* Binv, const float* b,
                            const float* Ax, float* p, float* x, float alpha, float beta, int first, hipStream_t s) {
  const size_t lds = sizeof(float) * size_t(L.nmax) * L.nmax * L.nmax;
  hipLaunchKernelGGL(block_cheb_bf16_kernel, dim3(unsigned(L.n_elem)), dim3(kBS), lds, s, L, boff, Binv, b, Ax, p,
                     x, alpha, beta, first);
}

// waves per element: one on levels with enough elements to fill the chip, more (up to 8) on
// small levels, where each wave's sequence of groups would otherwise set the time
// waves per element: doubled while every wave keeps at least 3 of the element's column blocks,
// or while the grid holds fewer than 8192 waves (small levels), never past 8 waves or half the
// column blocks (measured on blocks of 64, 125, 216 and 343 rows)
inline int block_waves(long long n_elem, int nmax) {
  const int ncb = (nmax * nmax * nmax + kGroup - 1) / kGroup;
  int w = 1;
  while (w < 8 && 2 * w <= ncb && (n_elem * w < 8192 || 6 * w <= ncb)) w *= 2;
  return w;
}
template <typename T, typename S>
void launch_block_apply(const LevelView<T>& L, const long long* poff, const S* P, const T* r, T* z,
                        hipStream_t s) {
  const int w = block_waves(L.n_elem, L.nmax);
  const size_t lds = (1 + w) * sizeof(T) * size_t(L.nmax) * L.nmax * L.nmax;
  hipLaunchKernelGGL((block_sym_kernel<S, T, false>), dim3(unsigned(L.n_elem)), dim3(64 * w), lds, s, L, poff, P,
                     r, (const T*)nullptr, (T*)nullptr, z, T(0), T(0), 0);
}
template <typename T, typename S>
void launch_block_cheb(const LevelView<T>& L, const long long* poff, const S* P, const T* b, const T* Ax, T* p,
                       T* x, T alpha, T beta, int first, hipStream_t s) {
  const int w = block_waves(L.n_elem, L.nmax);
  const size_t lds = (1 + w) * sizeof(T) * size_t(L.nmax) * L.nmax * L.nmax;
  hipLaunchKernelGGL((block_sym_kernel<S, T, true>), dim3(unsigned(L.n_elem)), dim3(64 * w), lds, s, L, poff, P,
                     b, Ax, p, x, alpha, beta, first);
}
#define HPDG_BLOCK_INST(T, S)                                                                             \
  template void launch_block_apply<T, S>(const LevelView<T>&, const long long*, const S*, const T*, T*,  \
                                         hipStream_t);                                                    \
  template void launch_block_cheb<T, S>(const LevelView<T>&, const long long*, const S*, const T*,       \
                                        const T*, T*, T*, T, T, int, hipStream_t);
HPDG_BLOCK_INST(double, double)
HPDG_BLOCK_INST(float, float)
#undef HPDG_BLOCK_INST

void launch_check_blocks(const LevelView<double>& L, const long long* boff, const double* B, const double* dinv,
                         int* bad, hipStream_t s) {
  hipLaunchKernelGGL(check_blocks_kernel, dim3(unsigned(L.n_elem)), dim3(kBS), 0, s, L, boff, B, dinv, bad);
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
                        T beta, int first, hipStream_t s, T* xo) {
  hipLaunchKernelGGL(cheb_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, n, b, Ax, dinv, p, x, alpha,
                     beta, first, xo ? xo : x);
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
  template void launch_prolong_add<T>(const TransferView<T>&, const T*, T*, hipStream_t);       \
  template void launch_restrict<T>(const TransferView<T>&, const T*, T*, hipStream_t);          \
  template void launch_fill<T>(long long, T, T*, hipStream_t);                                  \
  template void launch_copy<T>(long long, const T*, T*, hipStream_t);                           \
  template void launch_axpby<T>(long long, T, const T*, T, T*, hipStream_t);                    \
  template void launch_cheb_update<T>(long long, const T*, const T*, const T*, T*, T*, T, T, int, \
                                      hipStream_t, T*);                                         \
  template void launch_dense_matvec<T>(int, const T*, const T*, T*, hipStream_t);           \
  template void launch_scale<T>(long long, const T*, const T*, T*, hipStream_t);               \
  template void launch_set_unit<T>(const LevelView<T>&, int, T, T*, hipStream_t);              \
  template void launch_gather_column<T>(const LevelView<T>&, int, const T*, const long long*, T*, \
                                        hipStream_t);
HPDG_INST(double)
HPDG_INST(float)
#undef HPDG_INST

}  // namespace hpdg
