// Device-side views of a level and the kernel launchers (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "host.hpp"

namespace hpdg {

// 1-D table offsets mirrored from OpTable (ints in device memory)
struct TabView {
  const int* off;        // [12][kMaxN + 1][kMaxQ + 1]
  const int* dg_off;     // [kMaxQ + 1]
  const int* w_off;      // [kMaxQ + 1]
  const int* dface_off;  // [kMaxN + 1]
  const int* gl_off;     // [kMaxQ + 1]: GL nodes
};

template <typename T>
struct LevelView {
  const ElemInfo* einfo;
  const MortarInfo* minfo;
  const int* fmlist;
  const MortarTask* mtask;  // mortars with an operator term (mortar kernel)
  long long n_mtask;
  const T* vgeo;
  const T* mgeo;
  const T* mcoef;  // w det J c at the GL points of elements with a mass term (null: no mass term)
  // element-centric apply, in the order of its element groups: face records (6 per element),
  // dof offsets, diagonal metric (3 per element), element ids; the face coefficient tuples
  // (S, sigma, mn, mo)
  const FaceLink* flink;
  const long long* fe_off;
  const long long* fe_toff;
  const T* fe_g;
  const int* fe_id;
  const T* fcoef;
  T* trace;        // face traces of every element (written by launch_traces before an apply)
  T* slot;         // lifted face terms per face-mortar list entry (written by launch_faces)
  const T* tab;
  TabView tv;
  long long n_elem;
  int nmax, qmax, qmmax;
  int self_only;  // 1: neighbour traces taken as zero (the element-diagonal blocks A_ee)
};

// a posteriori estimator (apply.hip): the host's point data (EstTables) on the device
struct EstVolume {
  const double* vol;        // per element, at its volume GL points: (W det J, 1 / det J, g)
  const long long* voff;    // per element: first scalar of its triples
  const double* he2p2;      // per element: h_e^2 p_e^2
};
struct EstFace {
  const double* face;       // per task, at its GL points: (h_m / p_m, g_D, S ratio, h_m ratio)
  const long long* foff;    // per task: first scalar of its pairs
  const int* tmortar;       // per task: the mortar's index
  double* out;              // per mortar: its part (mortars without a task keep their value)
};
// LDS of the volume kernel; the estimator of x on level L (L.mtask: one task per interior or
// Dirichlet mortar): face traces of x, volume parts into vol, mortar parts into ef.out (zeroed
// by the caller), eta2(e) into eta2
size_t est_lds_bytes(int nmax, int qmax);
void launch_estimator(const LevelView<double>& L, const double* x, const EstVolume& ev, const EstFace& ef,
                      long long n_tasks, double* vol, double* eta2, hipStream_t s);

// F += int g psi (the volume part of Eq. Fh2) on the elements of level L: g of the right-hand
// side kind with parameters P[nP] (device) at the GL points of each element's rule, the points
// mapped by the macro maps (macros: the mesh's macros, cells: its level-0 cells, on the device)
void launch_rhs_volume(const LevelView<double>& L, const Macro* macros, const Cell* cells, int kind,
                       const double* P, int nP, double* F, hipStream_t s);

template <typename T>
struct TransferView {
  const TransferInfo* tinfo;   // per fine element
  const int* cstart;           // per coarse element
  const int* clist;
  const T* tab;
  TabView tv;
  long long n_fine, n_coarse;
  int nmax;
};

size_t apply_lds_bytes(int nmax, int qmax, int qmmax, size_t scalar, bool compact);

// face traces of the elements list[0..count) (every element when list is null, count ignored):
// for each face, the values at its n^2 LGL nodes and the reference normal derivative there
// (read by the mortar kernel)
template <typename T>
void launch_traces(const LevelView<T>& L, const T* x, hipStream_t s, const int* list = nullptr,
                   long long count = 0);
// the face terms of every mortar from L.trace into L.slot (both sides of each mortar)
template <typename T>
void launch_faces(const LevelView<T>& L, hipStream_t s);
// the element kernel restricted to the elements elems[0..count) that share degree n - 1 and q
// GL points (the level's face slots written before)
template <typename T>
void launch_apply_bucket(const LevelView<T>& L, int n, int q, const int* elems, long long count, const T* x, T* y,
                         hipStream_t s);
// the fixed face-trace scratch of the no-allocation apply: its capacity in bytes; set-up of the
// current device's address (once per device, that device current; throws on failure); the
// address kept for a device (null before set-up)
size_t noalloc_scratch_bytes();
void init_noalloc_scratch(int device);
void* noalloc_scratch(int device);
// One Jacobi-scaled Chebyshev step fused behind the apply (Alg. 4 with M the element blocks or
// diag A): with r = b - A x, z = M^-1 r (packed FP64 / FP32 blocks, or the inverse diagonal),
// p = alpha z + beta p (first:
// alpha z), x += p, per element in the workgroup that computed (A x)_e. Every element's apply
// reads only its own x and the face traces written before the launch, so x is updated in place.
// The point-Jacobi Chebyshev step of Alg. 4 fused behind the element-centric apply:
// z = dinv (b - A x), p = alpha z + beta p (first: alpha z), xo = x + p.  xo must differ from x
// (neighbours read x during the launch).
template <typename T>
struct FastStep {
  const T* dinv;
  const T* b;
  T* p;
  T* xo;
  T alpha, beta;
  int first;
};
// One degree group of the element-centric apply: elements [start, start + count) of the
// level's group order, n LGL nodes per axis; nx == n: every interior neighbour has n nodes,
// nx > n: some has another number (at most nx); the 1-D mass and stiffness matrices and the
// end-point derivatives l_i'(-1), l_i'(+1) of the n-node basis.
template <typename T>
struct FastBucket {
  int n, nx;
  long long start, count;
  const T* M1;
  const T* K1;
  const T* df;
};
// The element-centric apply (fastapply.hip) of one group: y = (A x) on its elements (the face
// slots of their faces left to the mortar kernel written before), or the fused step st.  The
// groups of a level run in descending degree: each writes the face traces that the groups of
// lower degree read (faces between degrees).

template <typename T>
void launch_fast_apply(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, T* y, hipStream_t s);
template <typename T>
void launch_fast_cheb(const LevelView<T>& L, const FastBucket<T>& fb, const T* x, const FastStep<T>& st,
                      hipStream_t s);

template <typename T>
struct BlockStep {
  const T* dinv;          // non-null: point Jacobi (z = dinv r) instead of the element blocks
  const long long* poff;  // packed block offset of each element (scalars)
  const T* P;             // packed inverse blocks
  const T* b;
  T* p;
  T* x;
  T* trace_out;  // non-null: the face traces of the updated x are written here (the launch reads
                 // L.trace, so the two must differ)
  T alpha, beta;
  int first;
  T* xo;         // non-null: the updated x is written here instead of in place
};
// whether the elements of one bucket (degree n - 1, q GL points) can take the fused step: the
// compact apply layout (n^3 <= 512, q = n or n + 1)
bool apply_block_fusable(int n, int q);
// the element kernel and the step for the elements elems[0..count) of one bucket; the level's
// face slots must hold the face terms of x (launch_faces after the traces of x)
template <typename T>
void launch_apply_block_cheb(const LevelView<T>& L, int n, int q, const int* elems, long long count, const T* x,
                             const BlockStep<T>& bs, hipStream_t s);
template <typename T>
void launch_prolong_add(const TransferView<T>& V, const T* uc, T* uf, hipStream_t s);
template <typename T>
void launch_restrict(const TransferView<T>& V, const T* rf, T* rc, hipStream_t s);

// vectors
template <typename T>
void launch_fill(long long n, T value, T* x, hipStream_t s);
template <typename T>
void launch_copy(long long n, const T* x, T* y, hipStream_t s);
// y = a x + b y
template <typename T>
void launch_axpby(long long n, T a, const T* x, T b, T* y, hipStream_t s);
// r = dinv (b - Ax) (dinv may be null; Ax null means x = 0); p = alpha r + beta p (first: p = alpha r);
// xo = x + p (xo null: x in place)
template <typename T>
void launch_cheb_update(long long n, const T* b, const T* Ax, const T* dinv, T* p, T* x, T alpha,
                        T beta, int first, hipStream_t s, T* xo = nullptr);
// y = a .* x
template <typename T>
void launch_scale(long long n, const T* a, const T* x, T* y, hipStream_t s);
void launch_convert_d2f(long long n, const double* x, float* y, hipStream_t s);
void launch_convert_f2d(long long n, const float* x, double* y, hipStream_t s);
// dense y = A x (row-major n x n)
template <typename T>
void launch_dense_matvec(int n, const T* A, const T* x, T* y, hipStream_t s);

// element-block Jacobi. Setup: the FP64 blocks of element e, column-major at boff[e], size
// (n_e^3)^2; column j of every block at once from an apply to e_j in every element (n^3 > j)
template <typename T>
void launch_set_unit(const LevelView<T>& L, int j, T value, T* x, hipStream_t s);
template <typename T>
void launch_gather_column(const LevelView<T>& L, int j, const T* y, const long long* boff, T* B,
                          hipStream_t s);
// bad[e] = 1 + first column of element e's gathered block that is not symmetric or whose
// diagonal differs from 1 / dinv; 0 when consistent
void launch_check_blocks(const LevelView<double>& L, const long long* boff, const double* B, const double* dinv,
                         int* bad, hipStream_t s);
// the lower triangles of the inverted blocks (column-major, B[c N + r], r >= c) packed at
// poff[e] (N (N + 1) / 2 scalars, panels of 64 rows, see kernels.hip) in storage type S
// (double or float)
template <typename S>
void launch_pack_blocks(const LevelView<double>& L, const long long* boff, const double* B, const long long* poff,
                        S* P, hipStream_t s);
// full bf16 copies of the inverted blocks (both triangles, column-major at boff[e]; bf16 held
// as uint16_t, rounded to nearest even from the FP32 value) and the FP32 Chebyshev step that
// reads them (same update as launch_block_cheb)
void launch_blocks_bf16_full(const LevelView<double>& L, const long long* boff, const double* B, uint16_t* Bh,
                             hipStream_t s);
void launch_block_cheb_bf16(const LevelView<float>& L, const long long* boff, const uint16_t* Binv, const float* b,
                            const float* Ax, float* p, float* x, float alpha, float beta, int first, hipStream_t s);
// z = Binv r per element (packed blocks, storage S, arithmetic T)
template <typename T, typename S>
void launch_block_apply(const LevelView<T>& L, const long long* poff, const S* P, const T* r, T* z,
                        hipStream_t s);
// r = Binv (b - Ax) per element (Ax null: x = 0); p = alpha r + beta p (first: alpha r); x += p
template <typename T, typename S>
void launch_block_cheb(const LevelView<T>& L, const long long* poff, const S* P, const T* b, const T* Ax, T* p,
                       T* x, T alpha, T beta, int first, hipStream_t s);

// deterministic reductions: out[0..k) = dots, via partials (kRedBlocks * k doubles)
constexpr int kRedBlocks = 512;
void launch_dot(long long n, const double* a, const double* b, double* partials, double* out,
                hipStream_t s);
// FCG (Alg. 2): dots v.r, v.w, v.q into out[0..3)
void launch_dot3(long long n, const double* v, const double* r, const double* w, const double* q,
                 double* partials, double* out, hipStream_t s);
// FCG scalars and updates; sc = device scalars (see kernels.hip); r.r partials -> sc
void launch_fcg_scalars(double* sc, int first, hipStream_t s);
void launch_fcg_update(long long n, const double* v, const double* w, double* d, double* q,
                       double* u, double* r, double* sc, double* partials, int first, hipStream_t s);

// Newton linearisation (newton.hip): per element, u at the volume GL points; N(u) (LGL test
// functions, may be null) and / or the Jacobian's mass coefficient (may be null). kind 0, 1:
// N integrand w det J beta (1 + alpha u)^-7, mass w det J 7 alpha beta (1 + alpha u)^-8, and
// *bad = 1 when 1 + alpha u <= 0 somewhere; kind 2 (star): w det J beta u^5, mass
// -5 w det J beta u^4 (wbeta = w det J beta)
void launch_nl_eval(const LevelView<double>& L, int kind, const double* u, const double* alpha,
                    const double* wbeta, double* N, double* mcoef, int* bad, hipStream_t s);
// dinv = 1 / (diag(A) + diag(mass form with L.mcoef))
template <typename T>
void launch_diag_mass(const LevelView<T>& L, const T* diagA, T* dinv, hipStream_t s);
// coarse state from the fine one: fine polynomial of the containing child at each coarse node
template <typename T>
void launch_inject(const TransferView<T>& V, const T* uf, T* uc, hipStream_t s);
// dense column-major n x n: lower_to_upper = 0: A = (A + A^T) / 2; 1: copy the lower triangle up
template <typename T>
void launch_symmetrize_dense(int n, T* A, int lower_to_upper, hipStream_t s);

}  // namespace hpdg
