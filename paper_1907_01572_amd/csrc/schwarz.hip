// gfx950 kernels of the additive Schwarz smoother (Sec. II.D, Alg. schwarz_smoother): the
// weighted local solves of every subdomain as dense mat-vecs with the stored inverses, and the
// sum of the weighted local corrections into the iterate.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "schwarz.hpp"

namespace hpdg {

namespace {

constexpr int kSwBS = 512;   // eight waves per workgroup
constexpr int kSwRows = 8;   // rows in flight per wave
constexpr int kSchwarzElems = 64;  // elements per subdomain in the assembly tables (kSchwarzMaxElems)

// row stride of the stored rows of a subdomain of m points in type T: m rounded up to the
// 16-byte vector width (2 doubles, 4 floats)
template <typename T>
__host__ __device__ inline int sw_stride(int m) {
  constexpr int vw = 16 / int(sizeof(T));
  return (m + vw - 1) / vw * vw;
}

// inverse of subdomain s (lower triangle, column-major m x m at P + pofs[b]) -> rows r < nw of
// W_s A_ss^-1 in type T, row-major with the stride sw_stride<T>(m) at minv + moff[b] (both
// triangles; the pad columns zero)
template <typename T>
__global__ void __launch_bounds__(256) schwarz_pack_kernel(int m, int b0, const double* __restrict__ P,
                                                         const long long* __restrict__ pofs,
                                                         const long long* __restrict__ moff,
                                                         const int* __restrict__ nw,
                                                         const long long* __restrict__ wofs,
                                                         const double* __restrict__ w, T* __restrict__ minv) {
  const int b = b0 + blockIdx.y;
  const int mp = sw_stride<T>(m);
  const double* Pb = P + pofs[b];
  const long long total = (long long)nw[b] * mp;
  T* out = minv + moff[b];
  const double* wb = w + wofs[b];
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int r = int(t / mp), k = int(t - (long long)r * mp);
    double v = 0.0;
    if (k < m) v = r >= k ? Pb[r + (long long)k * m] : Pb[k + (long long)r * m];
    out[t] = T(wb[r] * v);
  }
}

// setup: x[off(b) + j] = value for the elements b of one colour with more than j nodes
__global__ void __launch_bounds__(256) schwarz_units_kernel(const int* __restrict__ members, int cnt,
                                                          const long long* __restrict__ eoff,
                                                          const int* __restrict__ en3, int j, double value,
                                                          double* __restrict__ x) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt; t += gridDim.x * blockDim.x) {
    const int b = members[t];
    if (j < en3[b]) x[eoff[b] + j] = value;
  }
}

// setup: column j of the operator blocks of the elements b of one colour from y = A x (x the
// unit vectors of schwarz_units_kernel): slot k of b (0: b itself, 1 + t: its t-th coupled
// element a = adj[adj_start[b] + t]) holds the n3_a x n3_b block at blk + boff[sstart[b] + k],
// column-major: blk[boff[sstart[b] + k] + j n3_a + i] = y[off(a) + i]
__global__ void __launch_bounds__(256) schwarz_gather_kernel(const int* __restrict__ members,
                                                           const long long* __restrict__ adj_start,
                                                           const int* __restrict__ adj,
                                                           const long long* __restrict__ eoff,
                                                           const int* __restrict__ en3,
                                                           const long long* __restrict__ sstart,
                                                           const long long* __restrict__ boff, int j,
                                                           const double* __restrict__ y, double* __restrict__ blk) {
  const int b = members[blockIdx.x];
  const int k = blockIdx.y;
  const long long a0 = adj_start[b];
  if (k > adj_start[b + 1] - a0 || j >= en3[b]) return;
  const int a = k == 0 ? b : adj[a0 + k - 1];
  const int n3a = en3[a];
  double* dst = blk + boff[sstart[b] + k] + (long long)j * n3a;
  const double* src = y + eoff[a];
  for (int i = threadIdx.x; i < n3a; i += blockDim.x) dst[i] = src[i];
}

// setup: A_ss of the subdomains subs[b] (m points each), column-major at A + b m^2, from the
// operator blocks (at boff, n3_a x n3_b each) through the assembly tables; one workgroup per
// column
__global__ void __launch_bounds__(256) schwarz_assemble_kernel(int m, const int* __restrict__ subs,
                                                             const long long* __restrict__ goff,
                                                             const unsigned char* __restrict__ lel,
                                                             const short* __restrict__ loc,
                                                             const int* __restrict__ els,
                                                             const signed char* __restrict__ slot,
                                                             const int* __restrict__ en3,
                                                             const long long* __restrict__ sstart,
                                                             const long long* __restrict__ boff,
                                                             const double* __restrict__ blk,
                                                             double* __restrict__ A) {
  constexpr int K = kSchwarzElems;
  const int b = blockIdx.y, q = blockIdx.x;
  const int c = subs[b];
  const long long o = goff[c];
  const int eq = lel[o + q];
  const int* ec = els + K * (long long)c;
  const long long* bq = boff + sstart[ec[eq]];
  const int jq = loc[o + q];
  const signed char* sc = slot + (long long)K * K * c + K * eq;
  double* out = A + (long long)b * m * m + (long long)q * m;
  for (int p = threadIdx.x; p < m; p += blockDim.x) {
    const int lp = lel[o + p];
    const int k = sc[lp];
    out[p] = k < 0 ? 0.0 : blk[bq[k] + (long long)jq * en3[ec[lp]] + loc[o + p]];
  }
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static __device__ inline double dot(type a, type x) { return a.x * x.x + a.y * x.y; }
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static __device__ inline float dot(type a, type x) { return a.x * x.x + a.y * x.y + a.z * x.z + a.w * x.w; }
};

// workgroup (s, c): rows [c rpc, (c + 1) rpc) of subdomain s.  r_s = R_s r is staged in LDS
// (zero-padded to the row stride), then each wave takes kSwRows rows at a time, its lanes
// reading the rows in 16-byte vectors (2 doubles or 4 floats; coalesced, nontemporal: each row
// is streamed once per cycle), and reduces them across the wave
template <typename T>
__global__ void __launch_bounds__(kSwBS) schwarz_local_kernel(const T* __restrict__ r,
                                                            const int* __restrict__ gidx,
                                                            const long long* __restrict__ goff,
                                                            const long long* __restrict__ woff,
                                                            const long long* __restrict__ moff,
                                                            const T* __restrict__ minv,
                                                            T* __restrict__ d, int rpc) {
  typedef typename Vec16<T>::type V;
  constexpr int vw = 16 / int(sizeof(T));
  extern __shared__ double2 lds2[];  // 16-byte aligned
  T* rs = reinterpret_cast<T*>(lds2);
  const int s = blockIdx.x;
  const long long g0 = goff[s];
  const int m = int(goff[s + 1] - g0);
  const int mp = sw_stride<T>(m);
  const long long w0 = woff[s];
  const int nw = int(woff[s + 1] - w0);
  const int row_begin = blockIdx.y * rpc;
  const int row_end = min(nw, row_begin + rpc);
  if (row_begin >= row_end) return;  // the whole workgroup: no barrier is skipped by part of it
  for (int k = threadIdx.x; k < mp; k += kSwBS) rs[k] = k < m ? r[gidx[g0 + k]] : T(0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const V* rsv = reinterpret_cast<const V*>(rs);
  const T* M = minv + moff[s];
  const int nv = mp / vw;
  for (int row = row_begin + wave * kSwRows; row < row_end; row += (kSwBS / 64) * kSwRows) {
    const V* Mr[kSwRows];
#pragma unroll
    for (int q = 0; q < kSwRows; ++q)  // rows past the end read the last row; their sums are dropped
      Mr[q] = reinterpret_cast<const V*>(M + (long long)min(row + q, row_end - 1) * mp);
    T acc[kSwRows];
#pragma unroll
    for (int q = 0; q < kSwRows; ++q) acc[q] = T(0);
    for (int k = lane; k < nv; k += 64) {
      const V x = rsv[k];
#pragma unroll
      for (int q = 0; q < kSwRows; ++q) acc[q] += Vec16<T>::dot(__builtin_nontemporal_load(Mr[q] + k), x);
    }
#pragma unroll
    for (int q = 0; q < kSwRows; ++q)
      for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
#pragma unroll
    for (int q = 0; q < kSwRows; ++q)
      if (lane == q && row + q < row_end) d[w0 + row + q] = acc[q];
  }
}

// x_i += sum over the subdomains holding dof i (in subdomain order) of their weighted corrections
template <typename T>
__global__ void __launch_bounds__(256) schwarz_scatter_kernel(long long n, const long long* __restrict__ ptr,
                                                            const int* __restrict__ list,
                                                            const T* __restrict__ d, T* __restrict__ x) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  T acc = T(0);
  for (long long k = ptr[i]; k < ptr[i + 1]; ++k) acc += d[list[k]];
  x[i] += acc;
}

}  // namespace

template <typename T>
void launch_schwarz_pack(int m, int count, const double* P, const long long* pofs, const long long* moff,
                         const int* nw, const long long* wofs, const double* w, T* minv, hipStream_t s) {
  for (int b0 = 0; b0 < count; b0 += 32768)  // grid y stays below its 65535 limit
    hipLaunchKernelGGL(schwarz_pack_kernel<T>, dim3(64, unsigned(std::min(32768, count - b0))), dim3(256), 0, s, m,
                       b0, P, pofs, moff, nw, wofs, w, minv);
}

int schwarz_stride(int m, int scalar_bytes) { return scalar_bytes == 4 ? sw_stride<float>(m) : sw_stride<double>(m); }

void launch_schwarz_units(int cnt, const int* members, const long long* eoff, const int* en3, int j, double value,
                          double* x, hipStream_t s) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(schwarz_units_kernel, dim3(unsigned(std::min(4096, (cnt + 255) / 256))), dim3(256), 0, s,
                     members, cnt, eoff, en3, j, value, x);
}

void launch_schwarz_gather(int cnt, int max_slots, const int* members, const long long* adj_start, const int* adj,
                           const long long* eoff, const int* en3, const long long* sstart, const long long* boff, int j,
                           const double* y, double* blk, hipStream_t s) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(schwarz_gather_kernel, dim3(unsigned(cnt), unsigned(max_slots)), dim3(256), 0, s, members,
                     adj_start, adj, eoff, en3, sstart, boff, j, y, blk);
}

void launch_schwarz_assemble(int m, int cnt, const int* subs, const long long* goff, const unsigned char* lel,
                             const short* loc, const int* els, const signed char* slot, const int* en3,
                             const long long* sstart, const long long* boff, const double* blk, double* A,
                             hipStream_t s) {
  for (int b0 = 0; b0 < cnt; b0 += 32768)  // grid y stays below its 65535 limit
    hipLaunchKernelGGL(schwarz_assemble_kernel, dim3(unsigned(m), unsigned(std::min(32768, cnt - b0))), dim3(256), 0,
                       s, m, subs + b0, goff, lel, loc, els, slot, en3, sstart, boff, blk, A + (long long)b0 * m * m);
}

template <typename T>
void launch_schwarz_local(int n_sub, int max_m, int max_nw, const T* r, const int* gidx, const long long* goff,
                          const long long* woff, const long long* moff, const T* minv, T* d, hipStream_t s) {
  if (n_sub <= 0 || max_nw <= 0) return;
  // split the rows of each subdomain over several workgroups when there are few subdomains:
  // about 2048 workgroups (8 per CU), chunks of whole wave passes
  const int pass = (kSwBS / 64) * kSwRows;
  int chunks = std::max(1, std::min((2048 + n_sub - 1) / n_sub, (max_nw + pass - 1) / pass));
  chunks = std::min(chunks, 65535);
  int rpc = (max_nw + chunks - 1) / chunks;
  rpc = (rpc + pass - 1) / pass * pass;
  chunks = (max_nw + rpc - 1) / rpc;
  const size_t lds = size_t(sw_stride<T>(max_m)) * sizeof(T);
  hipLaunchKernelGGL(schwarz_local_kernel<T>, dim3(unsigned(n_sub), unsigned(chunks)), dim3(kSwBS), lds, s, r, gidx,
                     goff, woff, moff, minv, d, rpc);
}

template <typename T>
void launch_schwarz_scatter(long long n, const long long* ptr, const int* list, const T* d, T* x, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(schwarz_scatter_kernel<T>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, n, ptr, list, d,
                     x);
}

#define HPDG_SW_INST(T)                                                                                        \
  template void launch_schwarz_pack<T>(int, int, const double*, const long long*, const long long*, const int*,  \
                                       const long long*, const double*, T*, hipStream_t);                        \
  template void launch_schwarz_local<T>(int, int, int, const T*, const int*, const long long*, const long long*, \
                                        const long long*, const T*, T*, hipStream_t);                          \
  template void launch_schwarz_scatter<T>(long long, const long long*, const int*, const T*, T*, hipStream_t);
HPDG_SW_INST(double)
HPDG_SW_INST(float)
#undef HPDG_SW_INST

}  // namespace hpdg
