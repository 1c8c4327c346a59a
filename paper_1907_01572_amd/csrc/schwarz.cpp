// Host layout of the additive Schwarz smoother (Sec. II.D, Alg. schwarz_smoother,
// Eq. schwarz_weight): element-centred subdomains, their points and weights.
#include "../../include/hpdg.h"
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>

namespace hpdg {

namespace {

// C1 smoothstep from -1 to 1 and its sign limits outside [-1, 1]
double phi(double t) {
  if (t > 1.0) return 1.0;
  if (t < -1.0) return -1.0;
  const double t2 = t * t;
  return t * (15.0 - 10.0 * t2 + 3.0 * t2 * t2) / 8.0;
}

// 1-D weight w(xi) with overlap width delta; a closed side (domain boundary) keeps the plateau
double weight(double xi, double delta, bool lower_open, bool upper_open) {
  if (delta == 0.0) {
    const double lo = !lower_open ? 1.0 : (xi > -1.0 ? 1.0 : (xi == -1.0 ? 0.5 : 0.0));
    const double hi = !upper_open ? 1.0 : (xi < 1.0 ? 1.0 : (xi == 1.0 ? 0.5 : 0.0));
    return lo * hi;
  }
  const double a = lower_open ? phi((xi + 1.0) / delta) : 1.0;
  const double b = upper_open ? phi((xi - 1.0) / delta) : -1.0;
  return 0.5 * (a - b);
}

}  // namespace

void schwarz_layout(const MacroMesh& mm, const LevelHost& L, int n_overlap, SchwarzLayout& out) {
  const int E = int(L.cells.size());
  if (E == 0) throw Error(HPDG_ERR_INVALID_MESH, "empty level");
  const int n = L.einfo[0].n;
  const int lev = L.cells[0].level;
  if (n_overlap < 1) throw Error(HPDG_ERR_INVALID_ARG, "Schwarz overlap must be at least 1");
  n_overlap = std::min(n_overlap, n - 1);  // a level of degree p holds at most p layers
  // scope: one degree, one refinement level, axis-aligned affine boxes
  std::vector<std::array<double, 3>> centre(E), half(E);
  for (int e = 0; e < E; ++e) {
    const Cell& c = L.cells[e];
    if (L.einfo[e].n != n || c.level != lev)
      throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs levels of one degree and one refinement level");
    if (mm.macros[c.macro].kind != 0)
      throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs affine elements");
    const double xi0[3] = {0.0, 0.0, 0.0};
    double x[3], J[3][3];
    cell_eval(mm, c, xi0, x, J);
    double big = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) big = std::max(big, std::fabs(J[i][j]));
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j)
        if (i != j && std::fabs(J[i][j]) > 1e-12 * big)
          throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs axis-aligned elements");
      if (!(J[i][i] > 0)) throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs axis-aligned elements");
      centre[e][i] = x[i];
      half[e][i] = J[i][i];
    }
  }
  // face neighbours: every mortar 1:1, the plus side on the opposite face, same tangential size
  std::vector<int>& F = out.fnb;
  F.assign(size_t(E) * 6, -1);
  for (const Mortar& m : L.mortars) {
    if (m.ep < 0) continue;
    if (m.sub != -1 || m.fp != (m.fm ^ 1) || m.orient != 0)
      throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs conforming faces in the elements' own frames");
    const int d = m.fm >> 1;
    for (int t = 0; t < 3; ++t)
      if (t != d && std::fabs(half[m.em][t] - half[m.ep][t]) > 1e-12 * half[m.em][t])
        throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing needs faces that match in size");
    F[size_t(m.em) * 6 + m.fm] = m.ep;
    F[size_t(m.ep) * 6 + m.fp] = m.em;
  }
  std::vector<double> xl(n), wl(n);
  gauss_lobatto(n, xl.data(), wl.data());
  const double delta = 1.0 + xl[n_overlap - 1];
  out.n = n;
  out.off.assign(size_t(E) + 1, 0);
  out.nw.assign(size_t(E), 0);
  out.elem.clear();
  out.loc.clear();
  out.w.clear();
  // step along face neighbours: the element on side o of c (o_d in {-1, 0, 1}), reached over the
  // axes in every order; -1 when none, an error when two orders disagree
  auto step = [&](int e, int d, int s) { return e < 0 ? -1 : F[size_t(e) * 6 + 2 * d + (s > 0 ? 1 : 0)]; };
  for (int c = 0; c < E; ++c) {
    bool open_lo[3], open_hi[3];
    for (int d = 0; d < 3; ++d) {
      open_lo[d] = F[size_t(c) * 6 + 2 * d] >= 0;
      open_hi[d] = F[size_t(c) * 6 + 2 * d + 1] >= 0;
    }
    std::vector<std::pair<int, std::array<int, 3>>> nb;  // (element, side)
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int o[3] = {ox, oy, oz};
          if (!ox && !oy && !oz) continue;
          int axes[3], na = 0;
          for (int d = 0; d < 3; ++d)
            if (o[d]) axes[na++] = d;
          int found = -1;
          bool any = false;
          std::array<int, 3> perm = {0, 1, 2};
          do {
            if (perm[0] >= na || (na > 1 && perm[1] >= na) || (na > 2 && perm[2] >= na)) continue;
            int e = c;
            for (int k = 0; k < na; ++k) e = step(e, axes[perm[k]], o[axes[perm[k]]]);
            if (e < 0) continue;
            if (any && e != found)
              throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing: inconsistent edge or corner neighbours");
            found = e;
            any = true;
          } while (std::next_permutation(perm.begin(), perm.end()));
          if (found >= 0) nb.push_back({found, {ox, oy, oz}});
        }
    std::sort(nb.begin(), nb.end());
    for (size_t k = 1; k < nb.size(); ++k)
      if (nb[k].first == nb[k - 1].first)
        throw Error(HPDG_ERR_UNSUPPORTED, "Schwarz smoothing: an element neighbours another on two sides");
    nb.insert(nb.begin(), {c, {0, 0, 0}});
    std::vector<int> el, lc;
    std::vector<double> wt;
    for (const auto& pr : nb) {
      const int e = pr.first;
      const std::array<int, 3>& o = pr.second;
      for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const double ext[3] = {xl[i] + 2.0 * o[0], xl[j] + 2.0 * o[1], xl[k] + 2.0 * o[2]};
            bool in = true;
            for (int d = 0; d < 3; ++d) in = in && std::fabs(ext[d]) <= 1.0 + delta + 1e-12;
            if (!in) continue;
            double w = 1.0;
            for (int d = 0; d < 3; ++d) w *= weight(ext[d], delta, open_lo[d], open_hi[d]);
            el.push_back(e);
            lc.push_back(i + n * (j + n * k));
            wt.push_back(w);
          }
    }
    // non-zero weights first (stable)
    int cnt = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t k = 0; k < el.size(); ++k)
        if ((wt[k] != 0.0) == (pass == 0)) {
          out.elem.push_back(el[k]);
          out.loc.push_back(lc[k]);
          out.w.push_back(wt[k]);
          if (pass == 0) ++cnt;
        }
    out.nw[c] = cnt;
    out.off[c + 1] = out.off[c] + (long long)el.size();
  }
}

void schwarz_assemble(const SchwarzLayout& lay, const std::vector<double>& blk, const std::vector<int>& subs, int m,
                      double* A) {
  const size_t n3 = size_t(lay.n) * lay.n * lay.n;
  parallel_for(subs.size(), [&](size_t b) {
    const int c = subs[b];
    const long long o = lay.off[c];
    // the subdomain's distinct elements and, per ordered pair, the block slot (or -1)
    std::vector<int> els, lel(static_cast<size_t>(m));
    for (int p = 0; p < m; ++p) {
      const int e = lay.elem[size_t(o + p)];
      size_t k = 0;
      while (k < els.size() && els[k] != e) ++k;
      if (k == els.size()) els.push_back(e);
      lel[size_t(p)] = int(k);
    }
    const size_t ne = els.size();
    std::vector<int> slot(ne * ne, -1);  // [column element][row element]
    for (size_t jb = 0; jb < ne; ++jb)
      for (size_t ia = 0; ia < ne; ++ia) {
        if (ia == jb) {
          slot[jb * ne + ia] = 0;
          continue;
        }
        for (int f = 0; f < 6; ++f)
          if (lay.fnb[size_t(els[jb]) * 6 + f] == els[ia]) slot[jb * ne + ia] = 1 + f;
      }
    double* Ab = A + b * size_t(m) * m;
    for (int q = 0; q < m; ++q) {
      const size_t eq = size_t(lel[size_t(q)]);
      const size_t col = (size_t(els[eq]) * 7) * n3 * n3 + size_t(lay.loc[size_t(o + q)]) * n3;
      for (int p = 0; p < m; ++p) {
        const int k = slot[eq * ne + size_t(lel[size_t(p)])];
        Ab[size_t(p) + size_t(q) * m] = k < 0 ? 0.0 : blk[col + size_t(k) * n3 * n3 + size_t(lay.loc[size_t(o + p)])];
      }
    }
  });
}

}  // namespace hpdg
