// gfx950 kernels of the additive Schwarz smoother (Sec. II.D, Alg. schwarz_smoother): the
// weighted local solves of every subdomain as dense mat-vecs with the stored inverses, and the
// sum of the weighted local corrections into the iterate.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "schwarz.hpp"

namespace hpdg {

namespace {

constexpr int kSwBS = 256;  // four waves per subdomain

// inverse of subdomain s (lower triangle, column-major m x m at P + pofs[b]) -> rows r < nw of
// W_s A_ss^-1, row-major at minv + moff[b] (both triangles)
__global__ void __launch_bounds__(kSwBS) schwarz_pack_kernel(int m, int b0, const double* __restrict__ P,
                                                           const long long* __restrict__ pofs,
                                                           const long long* __restrict__ moff,
                                                           const int* __restrict__ nw,
                                                           const long long* __restrict__ wofs,
                                                           const double* __restrict__ w,
                                                           double* __restrict__ minv) {
  const int b = b0 + blockIdx.y;
  const double* Pb = P + pofs[b];
  const long long total = (long long)nw[b] * m;
  double* out = minv + moff[b];
  const double* wb = w + wofs[b];
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int r = int(t / m), k = int(t - (long long)r * m);
    const double v = r >= k ? Pb[r + (long long)k * m] : Pb[k + (long long)r * m];
    out[t] = wb[r] * v;
  }
}

// one workgroup per subdomain: r_s = R_s r into LDS, then d_s = W_s A_ss^-1 r_s, one wavefront
// per row (lanes along the row: coalesced reads of the stored rows), reduced across the wave
__global__ void __launch_bounds__(kSwBS) schwarz_local_kernel(const double* __restrict__ r,
                                                            const int* __restrict__ gidx,
                                                            const long long* __restrict__ goff,
                                                            const long long* __restrict__ woff,
                                                            const long long* __restrict__ moff,
                                                            const double* __restrict__ minv,
                                                            double* __restrict__ d) {
  extern __shared__ double rs[];
  const int s = blockIdx.x;
  const long long g0 = goff[s];
  const int m = int(goff[s + 1] - g0);
  const long long w0 = woff[s];
  const int nw = int(woff[s + 1] - w0);
  for (int k = threadIdx.x; k < m; k += kSwBS) rs[k] = r[gidx[g0 + k]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* M = minv + moff[s];
  for (int row = wave; row < nw; row += kSwBS / 64) {
    const double* Mr = M + (long long)row * m;
    double acc = 0.0;
    for (int k = lane; k < m; k += 64) acc += Mr[k] * rs[k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) d[w0 + row] = acc;
  }
}

// x_i += sum over the subdomains holding dof i (in subdomain order) of their weighted corrections
__global__ void __launch_bounds__(kSwBS) schwarz_scatter_kernel(long long n, const long long* __restrict__ ptr,
                                                              const int* __restrict__ list,
                                                              const double* __restrict__ d,
                                                              double* __restrict__ x) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (long long k = ptr[i]; k < ptr[i + 1]; ++k) acc += d[list[k]];
  x[i] += acc;
}

}  // namespace

void launch_schwarz_pack(int m, int count, const double* P, const long long* pofs, const long long* moff,
                         const int* nw, const long long* wofs, const double* w, double* minv, hipStream_t s) {
  for (int b0 = 0; b0 < count; b0 += 32768)  // grid y stays below its 65535 limit
    hipLaunchKernelGGL(schwarz_pack_kernel, dim3(64, unsigned(std::min(32768, count - b0))), dim3(kSwBS), 0, s, m,
                       b0, P, pofs, moff, nw, wofs, w, minv);
}

void launch_schwarz_local(int n_sub, int max_m, const double* r, const int* gidx, const long long* goff,
                          const long long* woff, const long long* moff, const double* minv, double* d,
                          hipStream_t s) {
  if (n_sub <= 0) return;
  hipLaunchKernelGGL(schwarz_local_kernel, dim3(n_sub), dim3(kSwBS), size_t(max_m) * sizeof(double), s, r, gidx,
                     goff, woff, moff, minv, d);
}

void launch_schwarz_scatter(long long n, const long long* ptr, const int* list, const double* d, double* x,
                            hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(schwarz_scatter_kernel, dim3(unsigned((n + kSwBS - 1) / kSwBS)), dim3(kSwBS), 0, s, n, ptr,
                     list, d, x);
}

}  // namespace hpdg
