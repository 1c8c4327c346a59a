// Host layout of the additive Schwarz smoother (Sec. II.D, Alg. schwarz_smoother,
// Eq. schwarz_weight): element-centred subdomains, their points and weights.
#include "../../include/hpdg.h"
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstdlib>
#include <unordered_map>

namespace hpdg {

namespace {

// C1 smoothstep from -1 to 1 and its sign limits outside [-1, 1]
double phi(double t) {
  if (t > 1.0) return 1.0;
  if (t < -1.0) return -1.0;
  const double t2 = t * t;
  return t * (15.0 - 10.0 * t2 + 3.0 * t2 * t2) / 8.0;
}

// one transition of the weight: phi(t / delta), or its limit sgn(t) for delta = 0
double edge(double t, double delta) {
  if (delta == 0.0) return t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0);
  return phi(t / delta);
}

// 1-D weight w(xi) with the overlap widths dlo (lower side) and dhi (upper side); a closed side
// (domain boundary) keeps the plateau
double weight(double xi, double dlo, double dhi, bool lower_open, bool upper_open) {
  const double a = lower_open ? edge(xi + 1.0, dlo) : 1.0;
  const double b = upper_open ? edge(xi - 1.0, dhi) : -1.0;
  return 0.5 * (a - b);
}

// affine map of a neighbour's reference coordinates into the centre's extended coordinates:
// ext[i] = sign[i] xi[perm[i]] + shift[i]
struct FaceMap {
  int perm[3];
  double sign[3], shift[3];
};

const FaceMap kIdentity = {{0, 1, 2}, {1.0, 1.0, 1.0}, {0.0, 0.0, 0.0}};

// the neighbour across face f (its face fb, orientation o from this face's coordinates to its
// own) seen from this element: its normal axis reversed or not so that the shared face lies at
// ext = +-1 on axis f / 2, its face axes permuted and flipped back by o
FaceMap face_map(int f, int fb, int o) {
  const int d = f >> 1, db = fb >> 1;
  const double sc = (f & 1) ? 1.0 : -1.0, sn = (fb & 1) ? 1.0 : -1.0;
  const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  const int u0 = db == 0 ? 1 : 0, u1 = db == 2 ? 1 : 2;
  FaceMap M = kIdentity;
  M.perm[d] = db;
  M.sign[d] = -sc * sn;
  M.shift[d] = 2.0 * sc;
  const int a0 = (o & 1) ? t1 : t0, a1 = (o & 1) ? t0 : t1;
  M.perm[a0] = u0;
  M.sign[a0] = (o & 2) ? -1.0 : 1.0;
  M.perm[a1] = u1;
  M.sign[a1] = (o & 4) ? -1.0 : 1.0;
  M.shift[a0] = M.shift[a1] = 0.0;
  return M;
}

// outer after inner
FaceMap compose(const FaceMap& outer, const FaceMap& inner) {
  FaceMap M;
  for (int i = 0; i < 3; ++i) {
    const int k = outer.perm[i];
    M.perm[i] = inner.perm[k];
    M.sign[i] = outer.sign[i] * inner.sign[k];
    M.shift[i] = outer.sign[i] * inner.shift[k] + outer.shift[i];
  }
  return M;
}

bool same_map(const FaceMap& a, const FaceMap& b) {
  for (int i = 0; i < 3; ++i)
    if (a.perm[i] != b.perm[i] || a.sign[i] != b.sign[i] || a.shift[i] != b.shift[i]) return false;
  return true;
}

uint64_t cell_key(const Cell& c) {
  return (uint64_t(c.macro) << 47) ^ (uint64_t(c.level) << 42) ^ (uint64_t(c.a[0]) << 28) ^
         (uint64_t(c.a[1]) << 14) ^ uint64_t(c.a[2]);
}

}  // namespace

namespace {

// per number of nodes n: the LGL nodes and the overlap width 1 + xi_(N_overlap - 1) (at most p
// layers: N_overlap <= n - 1); out.en / out.n set
void node_tables(const LevelHost& L, int n_overlap, SchwarzLayout& out, std::vector<std::vector<double>>& xln,
                 std::vector<double>& width) {
  const int E = int(L.cells.size());
  xln.assign(kMaxN + 1, std::vector<double>());
  width.assign(kMaxN + 1, 0.0);
  out.en.assign(size_t(E), 0);
  out.n = 0;
  for (int e = 0; e < E; ++e) {
    const int n = L.einfo[e].n;
    out.en[e] = n;
    out.n = std::max(out.n, n);
    if (!xln[n].empty()) continue;
    std::vector<double> wl(n);
    xln[n].resize(n);
    gauss_lobatto(n, xln[n].data(), wl.data());
    width[n] = 1.0 + xln[n][std::min(n_overlap, n - 1) - 1];
  }
}

// the elements coupled to each element by the operator (across interior mortars), sorted
void adjacency(const LevelHost& L, SchwarzLayout& out) {
  const size_t E = L.cells.size();
  std::vector<std::vector<int>> nb(E);
  for (const Mortar& m : L.mortars)
    if (m.ep >= 0 && m.ep != m.em) {
      nb[m.em].push_back(m.ep);
      nb[m.ep].push_back(m.em);
    }
  out.adj_start.assign(E + 1, 0);
  out.adj.clear();
  for (size_t e = 0; e < E; ++e) {
    std::sort(nb[e].begin(), nb[e].end());
    nb[e].erase(std::unique(nb[e].begin(), nb[e].end()), nb[e].end());
    out.adj.insert(out.adj.end(), nb[e].begin(), nb[e].end());
    out.adj_start[e + 1] = (long long)out.adj.size();
  }
}

// weights divided by their sum wherever it is not one; entries of each subdomain stably
// reordered with the non-zero weights first
void finish_layout(const LevelHost& L, std::vector<std::vector<int>>& el_all, std::vector<std::vector<int>>& lc_all,
                   std::vector<std::vector<double>>& wt_all, SchwarzLayout& out) {
  const int E = int(el_all.size());
  std::vector<double> total(size_t(L.ndof), 0.0);
  for (int c = 0; c < E; ++c)
    for (size_t k = 0; k < el_all[c].size(); ++k)
      total[size_t(L.einfo[el_all[c][k]].off + lc_all[c][k])] += wt_all[c][k];
  for (int c = 0; c < E; ++c)
    for (size_t k = 0; k < el_all[c].size(); ++k) {
      const double t = total[size_t(L.einfo[el_all[c][k]].off + lc_all[c][k])];
      if (std::fabs(t - 1.0) > 1e-12) wt_all[c][k] /= t;
    }
  out.off.assign(size_t(E) + 1, 0);
  out.nw.assign(size_t(E), 0);
  out.elem.clear();
  out.loc.clear();
  out.w.clear();
  for (int c = 0; c < E; ++c) {
    const std::vector<int>& el = el_all[c];
    int cnt = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t k = 0; k < el.size(); ++k)
        if ((wt_all[c][k] != 0.0) == (pass == 0)) {
          out.elem.push_back(el[k]);
          out.loc.push_back(lc_all[c][k]);
          out.w.push_back(wt_all[c][k]);
          if (pass == 0) ++cnt;
        }
    out.nw[c] = cnt;
    out.off[c + 1] = out.off[c] + (long long)el.size();
  }
}

// levels with 2:1 faces, on axis-aligned affine boxes: the extended coordinate of a point is its
// offset from e_c's centre in units of e_c's half-widths; the width of a cell of degree p and
// half-width h is delta_p h, each side of e_c taking the narrowest width, in its units, of e_c
// and the cells across that face; neighbours: the cells whose boxes touch e_c's, found within
// four face steps
void layout_boxes(const MacroMesh& mm, const LevelHost& L, int n_overlap, SchwarzLayout& out) {
  const int E = int(L.cells.size());
  std::vector<std::array<double, 3>> centre(E), half(E);
  for (int e = 0; e < E; ++e) {
    const Cell& c = L.cells[e];
    if (mm.macros[c.macro].kind != 0)
      throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing across 2:1 faces needs affine elements");
    const double xi0[3] = {0.0, 0.0, 0.0};
    double x[3], J[3][3];
    cell_eval(mm, c, xi0, x, J);
    double big = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) big = std::max(big, std::fabs(J[i][j]));
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j)
        if (i != j && std::fabs(J[i][j]) > 1e-12 * big)
          throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing across 2:1 faces needs axis-aligned elements");
      if (!(J[i][i] > 0)) throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing across 2:1 faces needs axis-aligned elements");
      centre[e][i] = x[i];
      half[e][i] = J[i][i];
    }
  }
  adjacency(L, out);
  std::vector<std::vector<double>> xln;
  std::vector<double> width;
  node_tables(L, n_overlap, out, xln, width);
  double hmin = std::numeric_limits<double>::infinity();
  for (int e = 0; e < E; ++e)
    for (int d = 0; d < 3; ++d) hmin = std::min(hmin, half[e][d]);
  const double tol = 1e-10 * hmin;
  std::vector<std::vector<int>> el_all(E), lc_all(E);
  std::vector<std::vector<double>> wt_all(E);
  parallel_for(size_t(E), [&](size_t ci) {
    const int c = int(ci);
    // candidates within four face steps, kept when the boxes touch
    std::vector<int> cand = {c};
    for (int step = 0; step < 4; ++step) {
      const size_t n0 = cand.size();
      for (size_t t = 0; t < n0; ++t)
        for (long long k = out.adj_start[cand[t]]; k < out.adj_start[cand[t] + 1]; ++k) cand.push_back(out.adj[k]);
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    }
    std::vector<int> touch;
    for (int e : cand) {
      if (e == c) continue;
      bool t = true;
      for (int d = 0; d < 3; ++d) t = t && std::fabs(centre[e][d] - centre[c][d]) - (half[e][d] + half[c][d]) <= tol;
      if (t) touch.push_back(e);
    }
    const double dc = width[out.en[c]];
    bool open_lo[3] = {false, false, false}, open_hi[3] = {false, false, false};
    double d_lo[3] = {0, 0, 0}, d_hi[3] = {0, 0, 0};
    for (int e : touch)
      for (int d = 0; d < 3; ++d) {
        // across a face of e_c: touching along d, overlapping with positive extent on the others
        bool face = std::fabs(std::fabs(centre[e][d] - centre[c][d]) - (half[e][d] + half[c][d])) <= tol;
        for (int t = 0; t < 3; ++t)
          if (t != d) face = face && std::fabs(centre[e][t] - centre[c][t]) - (half[e][t] + half[c][t]) < -tol;
        if (!face) continue;
        const double w = std::min(dc, width[out.en[e]] * half[e][d] / half[c][d]);
        if (centre[e][d] < centre[c][d]) {
          d_lo[d] = open_lo[d] ? std::min(d_lo[d], w) : w;
          open_lo[d] = true;
        } else {
          d_hi[d] = open_hi[d] ? std::min(d_hi[d], w) : w;
          open_hi[d] = true;
        }
      }
    touch.insert(touch.begin(), c);
    for (int e : touch) {
      const int n = out.en[e];
      const std::vector<double>& xl = xln[n];
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const double xi[3] = {xl[i], xl[j], xl[k]};
            double ext[3];
            bool in = true;
            for (int d = 0; d < 3; ++d) {
              ext[d] = (centre[e][d] + half[e][d] * xi[d] - centre[c][d]) / half[c][d];
              if (std::fabs(std::fabs(ext[d]) - 1.0) <= 1e-12) ext[d] = ext[d] > 0 ? 1.0 : -1.0;  // on e_c's faces
              const double bound = 1.0 + (ext[d] > 1.0 ? d_hi[d] : (ext[d] < -1.0 ? d_lo[d] : 0.0));
              in = in && std::fabs(ext[d]) <= bound + 1e-12;
            }
            if (!in) continue;
            double w = 1.0;
            for (int d = 0; d < 3; ++d) w *= weight(ext[d], d_lo[d], d_hi[d], open_lo[d], open_hi[d]);
            el_all[c].push_back(e);
            lc_all[c].push_back(i + n * (j + n * k));
            wt_all[c].push_back(w);
          }
    }
  });
  finish_layout(L, el_all, lc_all, wt_all, out);
}

}  // namespace

void schwarz_layout(const MacroMesh& mm, const LevelHost& L, int n_overlap, SchwarzLayout& out) {
  const int E = int(L.cells.size());
  if (E == 0) throw Error(HPDG_ERR_INVALID_MESH, "empty level");
  const int lev = L.cells[0].level;
  if (n_overlap < 1) throw Error(HPDG_ERR_INVALID_ARG, "Schwarz overlap must be at least 1");
  // levels with several refinement levels (2:1 faces): the construction from positions (boxes)
  for (int e = 0; e < E; ++e)
    if (L.cells[e].level != lev) {
      layout_boxes(mm, L, n_overlap, out);
      return;
    }
  // one refinement level: faces that meet 1:1 (any macro maps, face orientations and degrees)
  for (const Mortar& m : L.mortars)
    if (m.ep >= 0 && m.sub != -1) throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs faces that meet 1:1");
  adjacency(L, out);
  std::unordered_map<uint64_t, int> index;
  index.reserve(size_t(E) * 2);
  for (int e = 0; e < E; ++e) index[cell_key(L.cells[e])] = e;
  // per element and face: the neighbour, its face and the orientation
  std::vector<int> F(size_t(E) * 6, -1);
  std::vector<int> FB(size_t(E) * 6, -1), FO(size_t(E) * 6, 0);
  for (int e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      Cell nb;
      int fb = 0, o = 0;
      if (!cell_across(mm, L.cells[e], f, nb, fb, o)) continue;
      auto it = index.find(cell_key(nb));
      if (it == index.end()) throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs faces that meet 1:1");
      F[size_t(e) * 6 + f] = it->second;
      FB[size_t(e) * 6 + f] = fb;
      FO[size_t(e) * 6 + f] = o;
    }
  std::vector<std::vector<double>> xln;
  std::vector<double> width;
  node_tables(L, n_overlap, out, xln, width);
  out.off.assign(size_t(E) + 1, 0);
  out.nw.assign(size_t(E), 0);
  out.elem.clear();
  out.loc.clear();
  out.w.clear();
  struct Nb {
    int e;
    int o[3];
    FaceMap M;
  };
  std::vector<std::vector<int>> el_all(E), lc_all(E);
  std::vector<std::vector<double>> wt_all(E);
  parallel_for(size_t(E), [&](size_t ci) {
    const int c = int(ci);
    // neighbours at every offset: the face paths in every order of the offset's axes; an offset
    // whose paths disagree (or that leads back to c or one of its face neighbours: three cells
    // around an edge) has none
    std::vector<Nb> nb;
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int off[3] = {ox, oy, oz};
          int axes[3], na = 0;
          for (int d = 0; d < 3; ++d)
            if (off[d]) axes[na++] = d;
          if (na == 0) continue;
          int found = -1;
          FaceMap fm = kIdentity;
          bool bad = false, any = false;
          int order[3] = {0, 1, 2};
          do {
            if (order[0] >= na || (na > 1 && order[1] >= na) || (na > 2 && order[2] >= na)) continue;
            int e = c;
            FaceMap M = kIdentity;
            for (int k = 0; k < na && e >= 0; ++k) {
              const int a = axes[order[k]];
              const int j = M.perm[a];
              const int face = 2 * j + (double(off[a]) * M.sign[a] > 0 ? 1 : 0);
              const size_t slot = size_t(e) * 6 + face;
              if (F[slot] < 0) {
                e = -1;
                break;
              }
              M = compose(M, face_map(face, FB[slot], FO[slot]));
              e = F[slot];
            }
            if (e < 0) continue;
            for (int d = 0; d < 3; ++d)
              if (M.shift[d] != 2.0 * off[d]) bad = true;
            if (any && (e != found || !same_map(M, fm))) bad = true;
            found = e;
            fm = M;
            any = true;
          } while (std::next_permutation(order, order + 3));
          if (!any || bad) continue;
          Nb x;
          x.e = found;
          for (int d = 0; d < 3; ++d) x.o[d] = off[d];
          x.M = fm;
          nb.push_back(x);
        }
    std::vector<int> faces;
    for (const Nb& x : nb)
      if (std::abs(x.o[0]) + std::abs(x.o[1]) + std::abs(x.o[2]) == 1) faces.push_back(x.e);
    std::vector<Nb> keep;
    for (const Nb& x : nb) {
      const bool edge = std::abs(x.o[0]) + std::abs(x.o[1]) + std::abs(x.o[2]) > 1;
      if (x.e == c || (edge && std::find(faces.begin(), faces.end(), x.e) != faces.end())) continue;
      keep.push_back(x);
    }
    std::stable_sort(keep.begin(), keep.end(), [](const Nb& a, const Nb& b) { return a.e < b.e; });
    for (size_t k = 1; k < keep.size(); ++k)
      if (keep[k].e == keep[k - 1].e)
        throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing: an element neighbours another on two sides");
    // per side: open (a face neighbour) and its overlap width, the narrower of the two cells'
    bool open_lo[3], open_hi[3];
    double d_lo[3], d_hi[3];
    for (int d = 0; d < 3; ++d) {
      const int lo = F[size_t(c) * 6 + 2 * d], hi = F[size_t(c) * 6 + 2 * d + 1];
      open_lo[d] = lo >= 0;
      open_hi[d] = hi >= 0;
      d_lo[d] = lo >= 0 ? std::min(width[out.en[c]], width[out.en[lo]]) : 0.0;
      d_hi[d] = hi >= 0 ? std::min(width[out.en[c]], width[out.en[hi]]) : 0.0;
    }
    Nb self;
    self.e = c;
    self.o[0] = self.o[1] = self.o[2] = 0;
    self.M = kIdentity;
    keep.insert(keep.begin(), self);
    std::vector<int>& el = el_all[c];
    std::vector<int>& lc = lc_all[c];
    std::vector<double>& wt = wt_all[c];
    for (const Nb& x : keep) {
      const int n = out.en[x.e];
      const std::vector<double>& xl = xln[n];
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const double xi[3] = {xl[i], xl[j], xl[k]};
            double ext[3];
            bool in = true;
            for (int d = 0; d < 3; ++d) {
              ext[d] = x.M.sign[d] * xi[x.M.perm[d]] + x.M.shift[d];
              const double bound = 1.0 + (ext[d] > 1.0 ? d_hi[d] : (ext[d] < -1.0 ? d_lo[d] : 0.0));
              in = in && std::fabs(ext[d]) <= bound + 1e-12;
            }
            if (!in) continue;
            double w = 1.0;
            for (int d = 0; d < 3; ++d) w *= weight(ext[d], d_lo[d], d_hi[d], open_lo[d], open_hi[d]);
            el.push_back(x.e);
            lc.push_back(i + n * (j + n * k));
            wt.push_back(w);
          }
    }
  });
  finish_layout(L, el_all, lc_all, wt_all, out);
}

void schwarz_tables(const SchwarzLayout& lay, std::vector<unsigned char>& lel, std::vector<int>& els,
                    std::vector<signed char>& slot) {
  const size_t E = lay.nw.size();
  constexpr int K = kSchwarzMaxElems;
  lel.assign(lay.elem.size(), 0);
  els.assign(E * K, -1);
  slot.assign(E * K * K, -1);
  parallel_for(E, [&](size_t c) {
    const long long o = lay.off[c], m = lay.off[c + 1] - o;
    int* ec = els.data() + c * K;
    int ne = 0;
    for (long long p = 0; p < m; ++p) {
      const int e = lay.elem[size_t(o + p)];
      int k = 0;
      while (k < ne && ec[k] != e) ++k;
      if (k == ne) {
        if (ne == K) throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz subdomain of more than 64 elements");
        ec[ne++] = e;
      }
      lel[size_t(o + p)] = static_cast<unsigned char>(k);
    }
    signed char* sc = slot.data() + c * K * K;
    for (int jb = 0; jb < ne; ++jb)
      for (int ia = 0; ia < ne; ++ia) {
        if (ia == jb) {
          sc[jb * K + ia] = 0;
          continue;
        }
        const long long a0 = lay.adj_start[ec[jb]], a1 = lay.adj_start[ec[jb] + 1];
        for (long long t = a0; t < a1; ++t)
          if (lay.adj[size_t(t)] == ec[ia]) sc[jb * K + ia] = static_cast<signed char>(1 + (t - a0));
      }
  });
}

}  // namespace hpdg
