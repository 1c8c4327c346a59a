// Per-level host tables (geometry, mortars, transfers, diagonal) built at upload time.
#pragma once

#include <algorithm>
#include <exception>
#include <mutex>
#include <system_error>
#include <thread>
#include <vector>

#include "host.hpp"

namespace hpdg {

struct DiscParams {
  double C = 10.0;
  int quad_extra = 1;
  int coef_kind = 0;
  double coef[4] = {0, 0, 0, 0};
  int mass_term = 0;  // levels carry a mass term c u v with c set per GL point (Newton)
  // tabulated coefficients (hpdg_set_coefficient): 0 none, 1 one value per element, 2 nodal
  // values (level-vector layout, LGL interpolant per element); the values of every level are
  // in LevelHost::kvals / cvals
  int kfield = 0;
  int cfield = 0;
  double robin_gamma = 0.0;  // k n.grad u + gamma u = g_R on Robin faces (macro face kind 3)
  int ec_mode = 0;           // element-centric apply: 0 by level (see build_level), 1 always, 2 never
};

// 1-D operator tables, indexed by (kind, n, q); every matrix is row-major [q][n].
struct OpTable {
  // GL_*: LGL basis of n nodes at q GL points (full interval, lower half, upper half);
  // PR_*: coarse basis of n nodes at the q fine LGL nodes (prolongation, same cell / child);
  // IN_*: fine basis of n nodes at the q coarse LGL nodes mapped into the child (injection)
  // MASS1 / STIFF1 (index (kind, n, n)): the exact 1-D mass and stiffness matrices of the LGL
  // basis, int l_i l_j and int l_i' l_j' over [-1, 1] (symmetric n x n);
  // PROJ (index (kind, m, n), n rows of m columns): the L2 projection of the m-node LGL basis
  // onto the n-node one (the interpolation at the n nodes when m <= n, where it is exact)
  enum Kind { GL_VAL = 0, GL_DER = 1, GLLO_VAL = 2, GLLO_DER = 3, GLHI_VAL = 4, GLHI_DER = 5,
              PR_FULL = 6, PR_LO = 7, PR_HI = 8, IN_FULL = 9, IN_LO = 10, IN_HI = 11,
              MASS1 = 12, STIFF1 = 13, PROJ = 14, NKIND = 15 };
  std::vector<double> data;
  std::vector<int> off;        // [NKIND][kMaxN + 1][kMaxQ + 1]
  std::vector<int> dg_off;     // GL collocation derivative [q][q], by q
  std::vector<int> w_off;      // GL weights, by q
  std::vector<int> gl_off;     // GL nodes, by q
  std::vector<int> dface_off;  // l_i'(-1) then l_i'(+1), by n
  int index(int kind, int n, int q) const { return off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q]; }
  void build();
};

struct LevelHost {
  std::vector<Cell> cells;
  std::vector<Mortar> mortars;
  std::vector<ElemInfo> einfo;
  std::vector<MortarInfo> minfo;
  std::vector<int> fmlist;       // (mortar << 1) | side, grouped per element face
  std::vector<MortarTask> mtask; // mortars with an operator term, both sides, for the mortar kernel
  std::vector<double> vgeo, mgeo;
  std::vector<double> diag;
  long long ndof = 0;
  long long nmq = 0;  // mass-coefficient scalars (sum of q^3 over elements with a mass term)
  long long ntrace = 0;  // face-trace scalars (12 n^2 per element)
  long long nslot = 0;   // lifted face-term scalars (2 n^2 per face-mortar list entry)
  int nmax = 0, qmax = 0, qmmax = 0;
  // Element-centric apply (fastapply.hip) for axis-aligned affine elements with constant k and
  // no mass term: fast[e]; per element face its link (6 per element, used for fast elements);
  // the distinct face coefficient tuples (S, sigma, mn, mo); fast elements grouped by n (fast_nx:
  // n when every interior neighbour has degree n too, else a bound > n on the neighbours' n,
  // which selects the mixed-degree kernel and sizes its scratch); the elements whose face traces
  // the mortar kernel reads (sides of the mortars it evaluates)
  std::vector<unsigned char> fast;
  std::vector<FaceLink> flink;       // group order (fast_elems), 6 per element
  std::vector<long long> fast_off;   // group order: dof offset
  std::vector<long long> fast_toff;  // group order: face-trace offset (faces to lower degrees)
  std::vector<double> fast_g;        // group order: G00, G11, G22
  std::vector<double> fcoef;
  std::vector<int> fast_n, fast_nx;
  std::vector<long long> fast_start;
  std::vector<int> fast_elems;
  std::vector<int> trace_elems;
  // the other elements grouped by (n, q): kernels are specialised per group
  std::vector<int> bucket_n, bucket_q;
  std::vector<long long> bucket_start;
  std::vector<int> bucket_elems;
  // prolongation from the next coarser level: one record per element of this level
  std::vector<TransferInfo> tinfo;
  // restriction gathers: for each coarser element, the elements of this level inside it
  std::vector<int> cstart, clist;
  // tabulated diffusion / mass coefficient of this level (DiscParams::kfield / cfield)
  std::vector<double> kvals, cvals;
};

bool kconst(const DiscParams& dp);
double coef_k(const DiscParams& dp, const double x[3]);
// k at the point x = Phi_e(xi) of element e of level L: the tabulated value (per element, or
// the element's nodal interpolant at xi) or the analytic coefficient at x
double k_point(const DiscParams& dp, const LevelHost& L, int e, const double xi[3], const double x[3]);
// the tabulated coefficients of the next coarser level: per element the mean over the cells
// inside each coarse cell, per node the injection of the fine field (each coarse LGL node takes
// the value of the fine polynomial of the child containing it; on a cut the lower child)
void coarsen_fields(const DiscParams& dp, const LevelHost& fine, LevelHost& coarse);
// w det J c at the volume GL points of every element (mass-coefficient layout) for the
// tabulated mass coefficient c of the level
void mass_table(const MacroMesh& mm, const DiscParams& dp, const LevelHost& L, std::vector<double>& wc);

// element map: x, J at element reference point xi
void cell_eval(const MacroMesh& mm, const Cell& c, const double xi[3], double x[3], double J[3][3]);
double det3(const double J[3][3]);
void inv3(const double J[3][3], double Ji[3][3]);

// f(i) for i in [0, n) on up to 16 host threads (contiguous ranges; every f(i) writes only its
// own outputs, so the result does not depend on the split).  The first exception thrown by any
// f is rethrown here after every thread has been joined; a thread that cannot be started
// leaves its range to the calling thread.
template <typename F>
void parallel_for(size_t n, F&& f) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = std::min<size_t>(std::min<size_t>(hw, 16), std::max<size_t>(1, n / 64));
  std::exception_ptr err;
  std::mutex mu;
  auto range = [&](size_t lo, size_t hi) {
    try {
      for (size_t i = lo; i < hi; ++i) f(i);
    } catch (...) {
      std::lock_guard<std::mutex> lock(mu);
      if (!err) err = std::current_exception();
    }
  };
  if (nt <= 1) {
    range(0, n);
  } else {
    std::vector<std::thread> pool;
    size_t started = 0;
    for (; started < nt; ++started) {
      try {
        pool.emplace_back(range, n * started / nt, n * (started + 1) / nt);
      } catch (const std::system_error&) {
        break;
      }
    }
    if (started < nt) range(n * started / nt, n);
    for (std::thread& th : pool) th.join();
  }
  if (err) std::rethrow_exception(err);
}

// fill einfo / minfo / fmlist / vgeo / mgeo for a level (cells set)
void build_level(const MacroMesh& mm, const DiscParams& dp, const OpTable& T, LevelHost& L);
// transfer records between a fine level and the next coarser one
void build_transfer(LevelHost& fine, const LevelHost& coarse);
// diagonal of the level operator (Jacobi smoothing)
void build_diagonal(const OpTable& T, LevelHost& L);

// physical points and w det J at the volume GL points of every element with a mass term,
// in the mass-coefficient layout (element mq offset, points a + q (b + q c))
void mass_points(const MacroMesh& mm, const LevelHost& L, std::vector<double>& x, std::vector<double>& wdet);

// alpha(x), beta(x) of the source beta (1 + alpha u)^-7: kind 0 puncture
// (P = [s, rows (cx, cy, cz, m, a)]), kind 1 quadratic manufactured (P = [alpha, C (27)])
void nl_coefficients(int kind, const std::vector<double>& P, const double x[3], double& alpha, double& beta);

// the boundary part of the right-hand side F_h (Eq. Fh2) on level 0 (Dirichlet, Neumann and
// Robin faces); the volume part int g psi is added on the device (launch_rhs_volume)
void assemble_rhs(const MacroMesh& mm, const DiscParams& dp, const OpTable& T, const LevelHost& L,
                  int kind, const std::vector<double>& params, std::vector<double>& F);

// the mortar kernel's record of mortar M (both sides' traces, maps, rule; slots unset)
MortarTask mortar_task(const LevelHost& L, const MortarInfo& M);

// Point data of the a posteriori estimator (Eqs. Eta2_*) on level L for the problem (kind, P).
// The integrands live on the physical grid mm; the integration weights, h_e and h_m on ``grid``
// (a fiducial grid of the same cells, Sec. II.E; mm itself when null).  Per element at its
// volume GL points (W det J_grid, 1 / det J, g) and h_e^2 p_e^2; one mortar-kernel task per
// interior or Dirichlet mortar with, at its GL points (mortar frame, a + q b),
// (h_m / p_m, g_D, S_grid / S, h_m / h_m,grid) (h_m as for the penalty from the physical grid,
// the first entry from ``grid``; p_m = max(p-, p+); g_D = 0 inside): the mortar kernel's w S and
// sigma times the last two are the fiducial grid's.
struct EstTables {
  std::vector<double> vol;
  std::vector<long long> voff;  // per element: first scalar of its (W det J, 1 / det J, g) triples
  std::vector<double> he2p2;
  std::vector<MortarTask> tasks;
  std::vector<int> task_mortar;
  std::vector<double> face;
  std::vector<long long> foff;  // per task: first scalar of its 4-tuples
};
void estimator_tables(const MacroMesh& mm, const MacroMesh* grid, const DiscParams& dp, const LevelHost& L,
                      int kind, const std::vector<double>& P, EstTables& out);

// the cell of the same level (and degree) across face f of c: its face fb and the orientation
// from c's face coordinates to its (swap | flip of the first | flip of the second axis);
// false on the boundary (topo.cpp)
bool cell_across(const MacroMesh& mm, const Cell& c, int f, Cell& nb, int& fb, int& orient);

// Additive Schwarz subdomains of a level (Sec. II.D, Alg. schwarz_smoother, Eq. schwarz_weight),
// one per element e_c, for levels of one refinement level whose faces all meet 1:1
// (HPDG_ERR_UNSUPPORTED otherwise; any macro maps, face orientations and degrees).  The neighbours
// at each offset o (o_d in {-1, 0, 1}) are found by stepping across faces in every order of
// the offset's axes, and their reference coordinates carried into e_c's extended coordinates
// by the composed face maps (xi_ext = xi + 2 o in e_c's frame); an offset whose paths disagree,
// or that leads back to e_c or a face neighbour (three cells around an edge), has none.  The
// overlap width of a degree p is delta_p = 1 + xi_(N_overlap - 1) of its LGL nodes (N_overlap at
// most p); each face of e_c takes the narrower of its two cells' widths (ragged subdomains where
// degrees differ).  The subdomain holds the points with |xi_ext| <= 1 + delta of the side they
// lie on, on every axis, each weighted by the product over the axes of
// w(xi) = (phi((xi + 1) / delta_lo) - phi((xi - 1) / delta_hi)) / 2; on a side of e_c without a
// neighbour (domain boundary) that side's phi term is replaced by its limit; where the weights
// covering a point do not sum to one (three cells around an edge, widths that differ around an
// edge) they are divided by their sum.  Entries of a subdomain: e_c's points, then the neighbours' by element and local index,
// and then stably reordered so that the entries with a non-zero weight come first.
struct SchwarzLayout {
  std::vector<long long> off;     // per subdomain: first entry (E + 1)
  std::vector<int> nw;            // per subdomain: entries with a non-zero weight
  std::vector<int> elem, loc;     // element and local dof index of each entry
  std::vector<double> w;          // weight of each entry
  std::vector<long long> adj_start;  // per element: first of the elements it is coupled to (E + 1)
  std::vector<int> adj;              // the elements coupled by the operator (across mortars), sorted
  std::vector<int> en;            // per element: LGL nodes per axis
  int n = 0;                      // the largest of them
};
void schwarz_layout(const MacroMesh& mm, const LevelHost& L, int n_overlap, SchwarzLayout& out);
// Assembly tables of the subdomains: per entry, the index of its element among the subdomain's
// elements (lel); per subdomain, those elements (els, kSchwarzMaxElems per subdomain, -1 past
// the last) and, per ordered pair (column element, row element), the operator block holding
// their coupling (slot, kSchwarzMaxElems^2 per subdomain: 0 the element itself, 1 + t its t-th
// coupled element in adj, -1 none: the pair is not coupled)
constexpr int kSchwarzMaxElems = 64;
void schwarz_tables(const SchwarzLayout& lay, std::vector<unsigned char>& lel, std::vector<int>& els,
                    std::vector<signed char>& slot);

// one-side mortar map: rows of the 1-D matrices along the own face axes
struct SideMap {
  int swap, flipA, flipB, halfA, halfB;  // half: 0 full, 1 lower, 2 upper
};
SideMap side_map(const MortarInfo& M, int side);

}  // namespace hpdg
