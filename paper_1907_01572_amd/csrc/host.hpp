// Host-side data structures of the hpdg library: 1-D rules, analytic maps, octree
// topology (mortars, multigrid hierarchy) and the per-level tables that are uploaded.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace hpdg {

constexpr int kMaxN = 16;        // p <= 15
constexpr int kMaxQ = 20;        // GL points per axis

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ---- 1-D rules (basis.cpp) ------------------------------------------------------
void gauss_legendre(int q, double* x, double* w);
void gauss_lobatto(int n, double* x, double* w);
// L[a*n + i] = l_i(y_a), D[a*n + i] = l_i'(y_a) for Lagrange polynomials on nodes x[n]
void lagrange_eval(int n, const double* x, int m, const double* y, double* L, double* D);

// ---- macro maps (geom.cpp) ------------------------------------------------------
struct Macro {
  int kind;
  double par[16];
};
// x(xi) and J[i][j] = dx_i/dxi_j of a macro at macro coordinates xi; zc picks the branch
// of a piecewise radial map (the cell centre's xi2)
void macro_eval(const Macro& M, const double xi[3], double zc, double x[3], double J[3][3]);

// ---- octree topology (topo.cpp) ----------------------------------------------------
struct Cell {
  int macro, level, a[3], p;
};

struct MacroMesh {
  std::vector<Macro> macros;
  std::vector<int> nbr, nbr_face, nbr_orient, bc;  // [6 m + f]
};

struct Mortar {
  int em, fm, ep, fp;   // minus (finer / lower index) side; ep = -1 on the boundary
  int orient;           // minus face coordinates -> plus face coordinates
  int sub;              // -1, or ia + 2 ib: minus face inside the coarser plus face
  int bc;               // boundary kind (0 interior)
};

std::vector<Mortar> find_mortars(const MacroMesh& mm, const std::vector<Cell>& cells);
// one coarsening step: false when nothing coarsens
bool coarsen_cells(const MacroMesh& mm, const std::vector<Cell>& fine, std::vector<Cell>& coarse);
// hp-adaptation (Alg. hpamr): action per cell 0 keep, 1 h-refine (8 children of the same
// degree), 2 p-refine (degree + 1, at most max_p); then 2:1 restoration.  out: the new cells,
// each old cell replaced in place by the cells inside it (children by their bits, x fastest);
// origin: the old cell each new cell lies in
void adapt_cells(const MacroMesh& mm, const std::vector<Cell>& cells, const signed char* action, int max_p,
                 std::vector<Cell>& out, std::vector<int>& origin);
// for each fine cell: coarse cell index and child bits (-1 when the cell is identical)
void parent_cells(const std::vector<Cell>& fine, const std::vector<Cell>& coarse,
                  std::vector<int>& parent, std::vector<int>& bits);

// ---- element / mortar records shared with the device -----------------------------
struct ElemInfo {
  long long off;     // dof offset
  long long vgeo;    // offset of the volume metric (in scalars)
  long long mq;      // offset of the mass coefficient w det J c at the GL points (q^3 values)
  long long toff;    // offset of the element's face traces (6 faces x [values n^2, normal derivatives n^2])
  long long soff;    // offset of the element's lifted face terms: one slot of 2 n^2 scalars per entry of
                     // its face-mortar list, in list order (the mortar kernel writes, the apply sums)
  int n, q;          // LGL nodes and GL points per axis
  int vmode;         // 0: constant metric (affine, 6 values), 1: per GL point (6 q^3 values)
  int mass;          // 1: the level carries a mass term c u v
  int fstart[6];     // first entry of face f in the face-mortar list
  int fcnt[6];       // mortars on face f (0: no operator term)
};

struct MortarInfo {
  int em, fm, ep, fp;
  int orient, sub, q, gmode;  // gmode 0: constant per mortar (8 values), 1: per point (8 q^2)
  int bc;
  int rq;                     // the face's own rule (before any raise to the volume rule's q);
                              // Dirichlet data are integrated with it
  long long geo;              // offset of the mortar metric (in scalars)
};

// one mortar with an operator term, as the mortar kernel reads it: both sides' traces in, both
// sides' lifted face terms out (side 1 only on interior mortars)
struct MortarTask {
  long long tr[2];            // each side's traces on the mortar's face (values n^2, normal derivatives n^2)
  long long slot[2];          // each side's output slot (value lift n^2, normal-derivative lift n^2)
  long long geo;              // offset of the mortar metric
  signed char n[2], f[2];     // each side's LGL nodes per axis and face (0 for a missing side)
  signed char q, gmode, interior, pad;
  unsigned char map[2];       // side maps: swap | flipA << 1 | flipB << 2 | halfA << 3 | halfB << 5
  int pad2;
};

// one face of an element of the element-centric apply (fastapply.hip)
struct FaceLink {
  long long nb;  // kind 1: the neighbour's dof offset, or (neighbour of higher degree) the offset
                 // of the face trace it writes (values nn^2, normal derivatives nn^2)
  int meta;      // kind | neighbour n << 2 | neighbour face << 7 | frame map << 10 (swap, flipA, flipB)
                 // | 1 << 13 when the neighbour has a lower degree (this side writes its face trace)
                 // kind 0: no operator term; 1: interior, both sides read here; 2: boundary
                 // (Dirichlet or Robin); 3: the mortar kernel's lifted terms (face slots)
  int coef;      // kinds 1, 2: index of (S, sigma, own and neighbour normal coefficient) in the
                 // level's face-coefficient table
};
constexpr int kFastMaxN = 8;  // element-centric apply: p <= 7

struct TransferInfo {         // one per fine element
  long long foff, coff;       // dof offsets in the fine and coarse level
  int nf, nc, bits;           // bits: -1 same cell, else child bits (x | y<<1 | z<<2)
  int pad;
};

}  // namespace hpdg
