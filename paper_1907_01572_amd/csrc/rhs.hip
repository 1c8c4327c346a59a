// Volume part of the right-hand side, F_psi += int g psi (Eq. Fh2), on the device: one
// workgroup per element maps its GL points through the macro map, evaluates W det J g there
// and applies the transposed LGL -> GL interpolation along the three axes.
#include "apply_common.hpp"
#include "device.hpp"
#include "maps.hpp"

namespace hpdg {

namespace {

constexpr int kRhsThreads = 128;

__global__ void __launch_bounds__(kRhsThreads) rhs_volume_kernel(LevelView<double> L, const Macro* __restrict__ macros,
                                                                 const Cell* __restrict__ cells, int kind,
                                                                 const double* __restrict__ P, int nP,
                                                                 double* __restrict__ F) {
  extern __shared__ unsigned char smem_raw[];
  const long long e = blockIdx.x;
  if (e >= L.n_elem) return;
  const ElemInfo I = L.einfo[e];
  const Cell c = cells[e];
  const Macro& M = macros[c.macro];
  const int n = I.n, q = I.q, QM = L.qmax;
  double* gq = reinterpret_cast<double*>(smem_raw);  // [c][b][a]
  double* t1 = gq + QM * QM * QM;                    // [c][b][i]
  double* t2 = t1 + QM * QM * L.nmax;                // [c][j][i]
  const double* B = tab(L, 0, n, q);
  const double* w = L.tab + L.tv.w_off[q];
  const double* eta = L.tab + L.tv.gl_off[q];
  for (int idx = threadIdx.x; idx < q * q * q; idx += blockDim.x) {
    const int a = idx % q, b = (idx / q) % q, cc = idx / (q * q);
    const double xi[3] = {eta[a], eta[b], eta[cc]};
    double x[3], J[3][3];
    cell_map(M.kind, M.par, c.level, c.a, xi, x, J);
    gq[idx] = w[a] * w[b] * w[cc] * det3x3(J) * rhs_source(kind, P, nP, x);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q * q * n; idx += blockDim.x) {
    const int i = idx % n, cb = idx / n;
    double s = 0;
    for (int a = 0; a < q; ++a) s += B[a * n + i] * gq[cb * q + a];
    t1[idx] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < q * n * n; idx += blockDim.x) {
    const int i = idx % n, j = (idx / n) % n, cc = idx / (n * n);
    double s = 0;
    for (int b = 0; b < q; ++b) s += B[b * n + j] * t1[(cc * q + b) * n + i];
    t2[idx] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n * n; idx += blockDim.x) {
    const int ji = idx % (n * n), k = idx / (n * n);
    double s = 0;
    for (int cc = 0; cc < q; ++cc) s += B[cc * n + k] * t2[cc * n * n + ji];
    F[I.off + idx] += s;
  }
}

}  // namespace

void launch_rhs_volume(const LevelView<double>& L, const Macro* macros, const Cell* cells, int kind,
                       const double* P, int nP, double* F, hipStream_t s) {
  if (L.n_elem == 0) return;
  const size_t lds = sizeof(double) * (size_t(L.qmax) * L.qmax * L.qmax + size_t(L.qmax) * L.qmax * L.nmax +
                                       size_t(L.qmax) * L.nmax * L.nmax);
  hipLaunchKernelGGL(rhs_volume_kernel, dim3(unsigned(L.n_elem)), dim3(kRhsThreads), lds, s, L, macros, cells, kind,
                     P, nP, F);
}

}  // namespace hpdg
