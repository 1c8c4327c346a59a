// Launchers of the additive Schwarz smoother's kernels (schwarz.hip; Sec. II.D,
// Alg. schwarz_smoother).
#pragma once

#include <hip/hip_runtime.h>

namespace hpdg {

// Setup: unit vectors x[off(b) + j] = value for the cnt elements ``members`` with n_b^3 > j (one
// colour of a distance-2 colouring of the operator's coupling graph), and column j of their
// operator blocks from y = A x: slot k of b (0: b, 1 + t: a = adj[adj_start[b] + t]) at
// blk + boff[sstart[b] + k], n3_a x n3_b column-major; max_slots bounds 1 + the coupled elements
// of any member; eoff: each element's dof offset, en3: its n^3
void launch_schwarz_units(int cnt, const int* members, const long long* eoff, const int* en3, int j, double value,
                          double* x, hipStream_t s);
void launch_schwarz_gather(int cnt, int max_slots, const int* members, const long long* adj_start, const int* adj,
                           const long long* eoff, const int* en3, const long long* sstart, const long long* boff, int j,
                           const double* y, double* blk, hipStream_t s);
// Setup: A_ss of the cnt subdomains subs[b] of m points each, column-major at A + b m^2, from the
// operator blocks through the tables of schwarz_tables (lel and loc per entry at goff[subs[b]],
// els 64 and slot 64 x 64 per subdomain; the slot of an element pair indexes the column
// element's blocks at boff[sstart[e] + slot])
void launch_schwarz_assemble(int m, int cnt, const int* subs, const long long* goff, const unsigned char* lel,
                             const short* loc, const int* els, const signed char* slot, const int* en3,
                             const long long* sstart, const long long* boff, const double* blk, double* A,
                             hipStream_t s);
// row stride of the stored rows of a subdomain of m points for scalars of scalar_bytes bytes: m
// rounded up to the 16-byte vector width (2 doubles, 4 floats)
int schwarz_stride(int m, int scalar_bytes);
// Setup: rows r < nw[b] of W_s A_ss^-1 for the count subdomains of size m whose inverses (lower
// triangles, column-major) lie at P + pofs[b], written row-major in type T with the row stride
// schwarz_stride(m, sizeof(T)) (zero pad) at minv + moff[b] (moff a multiple of the vector
// width); the weights of the rows at w + wofs[b].
template <typename T>
void launch_schwarz_pack(int m, int count, const double* P, const long long* pofs, const long long* moff,
                         const int* nw, const long long* wofs, const double* w, T* minv, hipStream_t s);
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
