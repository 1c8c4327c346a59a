// Launchers of the additive Schwarz smoother's kernels (schwarz.hip; Sec. II.D,
// Alg. schwarz_smoother).
#pragma once

#include <hip/hip_runtime.h>

namespace hpdg {

// Setup: rows r < nw[b] of W_s A_ss^-1 for the count subdomains of size m whose inverses (lower
// triangles, column-major) lie at P + pofs[b], written row-major with the even row stride
// m + (m & 1) (zero pad) at minv + moff[b] (moff even); the weights of the rows at w + wofs[b].
void launch_schwarz_pack(int m, int count, const double* P, const long long* pofs, const long long* moff,
                         const int* nw, const long long* wofs, const double* w, double* minv, hipStream_t s);
// Smoothing (T = double, or float for the FP32 V-cycle with FP32 copies of the rows): per
// subdomain s (entries goff[s] .. goff[s + 1] with global dofs gidx, the first
// woff[s + 1] - woff[s] of them weighted) d[woff[s] + r] = (W_s A_ss^-1 R_s r)_r; max_m is the
// largest subdomain (its entries are staged in LDS, at most 8190), max_nw the most weighted rows
template <typename T>
void launch_schwarz_local(int n_sub, int max_m, int max_nw, const T* r, const int* gidx, const long long* goff,
                          const long long* woff, const long long* moff, const T* minv, T* d, hipStream_t s);
// x_i += sum of d[list[k]], k in [ptr[i], ptr[i + 1])
template <typename T>
void launch_schwarz_scatter(long long n, const long long* ptr, const int* list, const T* d, T* x, hipStream_t s);

}  // namespace hpdg
