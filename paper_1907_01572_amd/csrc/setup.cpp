// Host-side setup of a level: FP64 geometry at GL points (Sec. II.A.5, Eqs. Jacobian and
// Surface-Jacobian), mortar metric and penalty (Eq. penaltyparameter), transfer records
// (Sec. II.D.6), the operator diagonal and the right-hand side (Eq. Fh2).
#include "setup.hpp"
#include "maps.hpp"

#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <exception>
#include <mutex>
#include <system_error>
#include <thread>

namespace hpdg {

// ---------------------------------------------------------------------------------
void OpTable::build() {
  off.assign(NKIND * (kMaxN + 1) * (kMaxQ + 1), -1);
  dg_off.assign(kMaxQ + 1, -1);
  w_off.assign(kMaxQ + 1, -1);
  gl_off.assign(kMaxQ + 1, -1);
  dface_off.assign(kMaxN + 1, -1);
  data.clear();
  double xn[kMaxQ + 1], wn[kMaxQ + 1], eta[kMaxQ + 1], wq[kMaxQ + 1], pts[kMaxQ + 1];
  std::vector<double> L(kMaxQ * kMaxQ), D(kMaxQ * kMaxQ);
  auto push = [&](int kind, int n, int q, const double* M) {
    off[(kind * (kMaxN + 1) + n) * (kMaxQ + 1) + q] = int(data.size());
    data.insert(data.end(), M, M + q * n);
  };
  for (int n = 2; n <= kMaxN; ++n) {
    gauss_lobatto(n, xn, wn);
    for (int q = 1; q <= kMaxQ; ++q) {
      gauss_legendre(q, eta, wq);
      for (int half = 0; half < 3; ++half) {
        for (int a = 0; a < q; ++a)
          pts[a] = half == 0 ? eta[a] : 0.5 * (eta[a] + (half == 1 ? -1.0 : 1.0));
        lagrange_eval(n, xn, q, pts, L.data(), D.data());
        push(GL_VAL + 2 * half, n, q, L.data());
        push(GL_DER + 2 * half, n, q, D.data());
      }
      if (q >= 2 && q <= kMaxN) {  // prolongation: rows at the LGL nodes of q points
        double xf[kMaxN + 1], wf[kMaxN + 1];
        gauss_lobatto(q, xf, wf);
        for (int half = 0; half < 3; ++half) {
          for (int a = 0; a < q; ++a)
            pts[a] = half == 0 ? xf[a] : 0.5 * (xf[a] + (half == 1 ? -1.0 : 1.0));
          lagrange_eval(n, xn, q, pts, L.data(), D.data());
          push(PR_FULL + half, n, q, L.data());
        }
        for (int half = 0; half < 3; ++half) {  // injection: child coordinate of a coarse node
          for (int a = 0; a < q; ++a) pts[a] = half == 0 ? xf[a] : 2.0 * xf[a] + (half == 1 ? 1.0 : -1.0);
          lagrange_eval(n, xn, q, pts, L.data(), D.data());
          push(IN_FULL + half, n, q, L.data());
        }
      }
    }
    double ends[2] = {-1.0, 1.0};
    lagrange_eval(n, xn, 2, ends, L.data(), D.data());
    dface_off[n] = int(data.size());
    data.insert(data.end(), D.data(), D.data() + 2 * n);
  }
  // exact 1-D mass and stiffness matrices (Gauss rule of n points: the integrands have degree
  // <= 2n - 2) and the projections between LGL bases of different sizes
  {
    double xm[kMaxN + 1], wm[kMaxN + 1];
    std::vector<double> Ln(kMaxN * kMaxN), Dn(kMaxN * kMaxN), Lm(kMaxN * kMaxN), Dm(kMaxN * kMaxN);
    std::vector<double> Mm(kMaxN * kMaxN), Km(kMaxN * kMaxN), C(kMaxN * kMaxN), P(kMaxN * kMaxN);
    for (int n = 2; n <= kMaxN; ++n) {
      gauss_lobatto(n, xn, wn);
      gauss_legendre(n, eta, wq);
      lagrange_eval(n, xn, n, eta, Ln.data(), Dn.data());
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double m = 0, k = 0;
          for (int a = 0; a < n; ++a) {
            m += wq[a] * Ln[a * n + i] * Ln[a * n + j];
            k += wq[a] * Dn[a * n + i] * Dn[a * n + j];
          }
          Mm[i * n + j] = m;
          Km[i * n + j] = k;
        }
      push(MASS1, n, n, Mm.data());
      push(STIFF1, n, n, Km.data());
      for (int m = 2; m <= kMaxN; ++m) {
        gauss_lobatto(m, xm, wm);
        if (m <= n) {
          // the m-node polynomials are of degree < n: their values at the n nodes
          lagrange_eval(m, xm, n, xn, P.data(), Dm.data());
        } else {
          // P = M_n^-1 C with C_ij = int l_i^(n) l_j^(m) (Gauss rule of m points: exact)
          gauss_legendre(m, eta, wq);
          lagrange_eval(n, xn, m, eta, Ln.data(), Dn.data());
          lagrange_eval(m, xm, m, eta, Lm.data(), Dm.data());
          for (int i = 0; i < n; ++i)
            for (int j = 0; j < m; ++j) {
              double c = 0;
              for (int a = 0; a < m; ++a) c += wq[a] * Ln[a * n + i] * Lm[a * m + j];
              C[i * m + j] = c;
            }
          // Cholesky of the (SPD) mass matrix, then one solve per column of C
          std::vector<double> R(Mm.begin(), Mm.begin() + n * n);
          for (int j = 0; j < n; ++j) {
            double d = R[j * n + j];
            for (int k = 0; k < j; ++k) d -= R[j * n + k] * R[j * n + k];
            R[j * n + j] = std::sqrt(d);
            for (int i = j + 1; i < n; ++i) {
              double v = R[i * n + j];
              for (int k = 0; k < j; ++k) v -= R[i * n + k] * R[j * n + k];
              R[i * n + j] = v / R[j * n + j];
            }
          }
          for (int j = 0; j < m; ++j) {
            double z[kMaxN + 1];
            for (int i = 0; i < n; ++i) {
              double v = C[i * m + j];
              for (int k = 0; k < i; ++k) v -= R[i * n + k] * z[k];
              z[i] = v / R[i * n + i];
            }
            for (int i = n - 1; i >= 0; --i) {
              double v = z[i];
              for (int k = i + 1; k < n; ++k) v -= R[k * n + i] * z[k];
              z[i] = v / R[i * n + i];
            }
            for (int i = 0; i < n; ++i) P[i * m + j] = z[i];
          }
        }
        push(PROJ, m, n, P.data());
      }
    }
  }
  for (int q = 1; q <= kMaxQ; ++q) {
    gauss_legendre(q, eta, wq);
    w_off[q] = int(data.size());
    data.insert(data.end(), wq, wq + q);
    gl_off[q] = int(data.size());
    data.insert(data.end(), eta, eta + q);
    if (q >= 2) {
      lagrange_eval(q, eta, q, eta, L.data(), D.data());
      dg_off[q] = int(data.size());
      data.insert(data.end(), D.data(), D.data() + q * q);
    } else {
      dg_off[q] = int(data.size());
      data.push_back(0.0);
    }
  }
}

// ---------------------------------------------------------------------------------
bool kconst(const DiscParams& dp) { return dp.coef_kind == 0 && dp.kfield == 0; }

namespace {

// value at reference point xi of the LGL interpolant of the n^3 nodal values u (x fastest)
double nodal_at(int n, const double* u, const double xi[3]) {
  double xn[kMaxN + 1], wn[kMaxN + 1], L[3][kMaxN + 1], D[kMaxN + 1];
  gauss_lobatto(n, xn, wn);
  for (int d = 0; d < 3; ++d) lagrange_eval(n, xn, 1, &xi[d], L[d], D);
  double v = 0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) {
      double r = 0;
      for (int i = 0; i < n; ++i) r += L[0][i] * u[(k * n + j) * n + i];
      v += L[2][k] * L[1][j] * r;
    }
  return v;
}

double field_point(int kind, const std::vector<double>& vals, const LevelHost& L, int e, const double xi[3]) {
  if (kind == 1) return vals[size_t(e)];
  const ElemInfo& I = L.einfo[e];
  return nodal_at(I.n, vals.data() + I.off, xi);
}

}  // namespace

double k_point(const DiscParams& dp, const LevelHost& L, int e, const double xi[3], const double x[3]) {
  if (dp.kfield) return field_point(dp.kfield, L.kvals, L, e, xi);
  return coef_k(dp, x);
}

void coarsen_fields(const DiscParams& dp, const LevelHost& fine, LevelHost& coarse) {
  if (!dp.kfield && !dp.cfield) return;
  std::vector<int> parent, bits;
  parent_cells(fine.cells, coarse.cells, parent, bits);
  const size_t Ec = coarse.cells.size();
  long long cdof = 0;
  std::vector<long long> coff(Ec);
  for (size_t K = 0; K < Ec; ++K) {
    coff[K] = cdof;
    const long long nc = coarse.cells[K].p + 1;
    cdof += nc * nc * nc;
  }
  auto coarsen = [&](int kind, const std::vector<double>& fv, std::vector<double>& cv) {
    if (kind == 1) {
      std::vector<double> cnt(Ec, 0.0);
      cv.assign(Ec, 0.0);
      for (size_t k = 0; k < fine.cells.size(); ++k) {
        cv[size_t(parent[k])] += fv[k];
        cnt[size_t(parent[k])] += 1.0;
      }
      for (size_t K = 0; K < Ec; ++K) cv[K] /= cnt[K];
      return;
    }
    cv.assign(size_t(cdof), 0.0);
    double xc[kMaxN + 1], wc[kMaxN + 1];
    for (size_t k = 0; k < fine.cells.size(); ++k) {
      const int K = parent[k], b = bits[k];
      const int nf = fine.cells[k].p + 1, nc = coarse.cells[K].p + 1;
      gauss_lobatto(nc, xc, wc);
      const double* u = fv.data() + fine.einfo[k].off;
      for (int c = 0; c < nc; ++c)
        for (int bb = 0; bb < nc; ++bb)
          for (int a = 0; a < nc; ++a) {
            const int idx[3] = {a, bb, c};
            double xi[3];
            bool own = true;
            for (int d = 0; d < 3; ++d) {
              const double t = xc[idx[d]];
              if (b < 0) {
                xi[d] = t;
              } else {
                const int bd = (b >> d) & 1;
                xi[d] = 2.0 * t - 2.0 * bd + 1.0;
                own = own && (bd == 0 ? t <= 0.0 : t > 0.0);
              }
            }
            if (own) cv[size_t(coff[K]) + (size_t(c) * nc + bb) * nc + a] = nodal_at(nf, u, xi);
          }
    }
  };
  if (dp.kfield) coarsen(dp.kfield, fine.kvals, coarse.kvals);
  if (dp.cfield) coarsen(dp.cfield, fine.cvals, coarse.cvals);
}

double coef_k(const DiscParams& dp, const double x[3]) {
  if (dp.coef_kind == 1) {
    double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    return r < dp.coef[0] ? dp.coef[1] : dp.coef[2];
  }
  return 1.0;
}

double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

void inv3(const double J[3][3], double Ji[3][3]) {
  const double d = det3(J);
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
}

void cell_eval(const MacroMesh& mm, const Cell& c, const double xi[3], double x[3], double J[3][3]) {
  const Macro& M = mm.macros[c.macro];
  cell_map(M.kind, M.par, c.level, c.a, xi, x, J);
}

namespace {

void face_ref(int f, double a, double b, double xi[3]) {
  const int d = f >> 1;
  const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
  xi[d] = (f & 1) ? 1.0 : -1.0;
  xi[t0] = a;
  xi[t1] = b;
}

void plus_coords(int orient, int sub, double s, double t, double& a, double& b) {
  a = (orient & 1) ? t : s;
  b = (orient & 1) ? s : t;
  if (orient & 2) a = -a;
  if (orient & 4) b = -b;
  if (sub >= 0) {
    a = 0.5 * (a + 2.0 * (sub & 1) - 1.0);
    b = 0.5 * (b + 2.0 * ((sub >> 1) & 1) - 1.0);
  }
}

}  // namespace

SideMap side_map(const MortarInfo& M, int side) {
  SideMap s{0, 0, 0, 0, 0};
  if (side == 1) {
    s.swap = M.orient & 1;
    s.flipA = (M.orient >> 1) & 1;
    s.flipB = (M.orient >> 2) & 1;
    s.halfA = M.sub < 0 ? 0 : 1 + (M.sub & 1);
    s.halfB = M.sub < 0 ? 0 : 1 + ((M.sub >> 1) & 1);
  }
  return s;
}

MortarTask mortar_task(const LevelHost& L, const MortarInfo& M) {
  MortarTask t{};
  t.geo = M.geo;
  t.q = (signed char)M.q;
  t.gmode = (signed char)M.gmode;
  t.interior = M.ep >= 0 ? 1 : 0;
  for (int sd = 0; sd < 1 + t.interior; ++sd) {
    const ElemInfo& O = L.einfo[size_t(sd ? M.ep : M.em)];
    const int f = sd ? M.fp : M.fm;
    const SideMap sm = side_map(M, sd);
    t.n[sd] = (signed char)O.n;
    t.f[sd] = (signed char)f;
    t.tr[sd] = O.toff + 2LL * f * O.n * O.n;
    t.slot[sd] = -1;
    t.map[sd] = (unsigned char)(sm.swap | (sm.flipA << 1) | (sm.flipB << 2) | (sm.halfA << 3) | (sm.halfB << 5));
  }
  return t;
}

void build_level(const MacroMesh& mm, const DiscParams& dp, const OpTable& T, LevelHost& L) {
  const size_t E = L.cells.size();
  L.mortars = find_mortars(mm, L.cells);
  const bool kc = kconst(dp);
  L.einfo.assign(E, ElemInfo{});
  L.vgeo.clear();
  L.nmq = 0;
  L.ntrace = 0;
  L.nmax = L.qmax = L.qmmax = 0;
  // elements: nodes and dof offsets (a nodal k is read through them), then the rule and metric
  // mode (the check for one value of k evaluates k at every GL point)
  long long off = 0;
  for (size_t e = 0; e < E; ++e) {
    const Cell& c = L.cells[e];
    if (c.p < 1 || c.p > kMaxN - 1) throw Error(-2, "degree outside [1, 15]");
    ElemInfo& I = L.einfo[e];
    I.n = c.p + 1;
    I.off = off;
    off += (long long)I.n * I.n * I.n;
  }
  std::vector<double> kel_of(E, 1.0);
  parallel_for(E, [&](size_t e) {
    const Cell& c = L.cells[e];
    ElemInfo& I = L.einfo[e];
    const bool affine = mm.macros[c.macro].kind == 0;
    // affine, constant k and no mass term: every volume integrand is integrated exactly by n points
    I.q = I.n + ((affine && kc && !dp.mass_term) ? 0 : dp.quad_extra);
    if (I.q > kMaxQ) throw Error(-2, "too many quadrature points");
    // constant metric: affine map and one value of k at every GL point of the element (k is
    // folded into the 6 stored values; the rule keeps its q points)
    double kel = 1.0;
    bool kflat = kc;
    if (affine && !kc) {
      double eta[kMaxQ + 1], wq[kMaxQ + 1];
      gauss_legendre(I.q, eta, wq);
      kflat = true;
      for (int cc = 0; cc < I.q && kflat; ++cc)
        for (int b = 0; b < I.q && kflat; ++b)
          for (int a = 0; a < I.q && kflat; ++a) {
            double xi[3] = {eta[a], eta[b], eta[cc]}, xp[3], Jp[3][3];
            cell_eval(mm, c, xi, xp, Jp);
            const double kv = k_point(dp, L, int(e), xi, xp);
            if (a == 0 && b == 0 && cc == 0) kel = kv;
            kflat = kv == kel;
          }
    }
    I.vmode = (affine && kflat) ? 0 : 1;
    I.mass = dp.mass_term ? 1 : 0;
    kel_of[e] = kel;
  });
  long long nv = 0;
  for (size_t e = 0; e < E; ++e) {
    ElemInfo& I = L.einfo[e];
    I.mq = L.nmq;
    if (I.mass) L.nmq += (long long)I.q * I.q * I.q;
    I.toff = L.ntrace;
    L.ntrace += 12LL * I.n * I.n;
    I.vgeo = nv;
    nv += I.vmode == 0 ? 6 : 6LL * I.q * I.q * I.q;
    L.nmax = std::max(L.nmax, I.n);
    L.qmax = std::max(L.qmax, I.q);
  }
  L.vgeo.assign(size_t(nv), 0.0);
  parallel_for(E, [&](size_t e) {
    const ElemInfo& I = L.einfo[e];
    const Cell& c = L.cells[e];
    double* out = L.vgeo.data() + I.vgeo;
    const int pr[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double x[3], J[3][3], Ji[3][3];
    if (I.vmode == 0) {
      double xi[3] = {0, 0, 0};
      cell_eval(mm, c, xi, x, J);
      const double dj = det3(J);
      if (!(dj > 0)) throw Error(-2, "non-positive Jacobian determinant");
      inv3(J, Ji);
      for (int m = 0; m < 6; ++m) {
        double g = 0;
        for (int i = 0; i < 3; ++i) g += Ji[pr[m][0]][i] * Ji[pr[m][1]][i];
        out[m] = dj * kel_of[e] * g;
      }
      return;
    }
    const int q = I.q, q3 = q * q * q;
    double eta[kMaxQ + 1], wq[kMaxQ + 1];
    gauss_legendre(q, eta, wq);
    for (int cc = 0; cc < q; ++cc)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          double xi[3] = {eta[a], eta[b], eta[cc]};
          cell_eval(mm, c, xi, x, J);
          const double dj = det3(J);
          if (!(dj > 0)) throw Error(-2, "non-positive Jacobian determinant");
          inv3(J, Ji);
          const double sc = wq[a] * wq[b] * wq[cc] * dj * k_point(dp, L, int(e), xi, x);
          const int idx = a + q * (b + q * cc);
          for (int m = 0; m < 6; ++m) {
            double g = 0;
            for (int i = 0; i < 3; ++i) g += Ji[pr[m][0]][i] * Ji[pr[m][1]][i];
            out[size_t(m) * q3 + idx] = sc * g;
          }
        }
  });
  L.ndof = off;
  // mortars: rule and metric mode, then the metric
  const size_t M = L.mortars.size();
  L.minfo.assign(M, MortarInfo{});
  L.mgeo.clear();
  std::vector<std::vector<int>> lists(E * 6);
  std::vector<double> kmt_of(M, 1.0), kpt_of(M, 1.0);
  std::vector<int> pm_of(M, 0);
  // each side's k at a mortar point: a tabulated k may jump across the mortar, so each side
  // takes its own element's value (an analytic k is single-valued: the minus side's value)
  auto side_k = [&](const Mortar& mt, double s_, double t_, double& km, double& kp) {
    const Cell& cm = L.cells[mt.em];
    double xim[3], xp[3], Jp[3][3];
    face_ref(mt.fm, s_, t_, xim);
    cell_eval(mm, cm, xim, xp, Jp);
    km = k_point(dp, L, mt.em, xim, xp);
    kp = km;
    if (mt.ep >= 0 && dp.kfield) {
      double a, b, xip[3], xq[3], Jq[3][3];
      plus_coords(mt.orient, mt.sub, s_, t_, a, b);
      face_ref(mt.fp, a, b, xip);
      cell_eval(mm, L.cells[mt.ep], xip, xq, Jq);
      kp = k_point(dp, L, mt.ep, xip, xq);
    }
  };
  parallel_for(M, [&](size_t mi) {
    const Mortar& mt = L.mortars[mi];
    MortarInfo& I = L.minfo[mi];
    I.em = mt.em; I.fm = mt.fm; I.ep = mt.ep; I.fp = mt.fp;
    I.orient = mt.orient; I.sub = mt.sub; I.bc = mt.bc; I.rq = 0;
    const Cell& cm = L.cells[mt.em];
    const bool interior = mt.ep >= 0;
    const bool robin = !interior && mt.bc == 3;
    if (!interior && mt.bc != 1 && !robin) {  // Neumann: no operator term
      I.q = 0; I.gmode = 0; I.geo = -1;
      return;
    }
    const int nm = cm.p + 1;
    const int np = interior ? L.cells[mt.ep].p + 1 : 0;
    const bool curved = mm.macros[cm.macro].kind != 0 ||
                        (interior && mm.macros[L.cells[mt.ep].macro].kind != 0);
    pm_of[mi] = std::max(nm, np) - 1;
    I.q = std::max(nm, np) + ((curved || !kc) ? dp.quad_extra : 0);
    if (I.q > kMaxQ) throw Error(-2, "too many mortar quadrature points");
    I.rq = I.q;
    // constant metric on a flat mortar where each side's k takes one value at all its points
    // (folded in)
    double kmt = 1.0, kpt = 1.0;
    bool kflat = kc;
    if (!curved && !kc) {
      double eta[kMaxQ + 1], wq[kMaxQ + 1];
      gauss_legendre(I.q, eta, wq);
      kflat = true;
      for (int pidx = 0; pidx < I.q * I.q && kflat; ++pidx) {
        double km, kp;
        side_k(mt, eta[pidx % I.q], eta[pidx / I.q], km, kp);
        if (pidx == 0) {
          kmt = km;
          kpt = kp;
        }
        kflat = km == kmt && kp == kpt;
      }
    }
    I.gmode = (curved || !kflat) ? 1 : 0;
    kmt_of[mi] = kmt;
    kpt_of[mi] = kpt;
  });
  long long ng = 0;
  for (size_t mi = 0; mi < M; ++mi) {
    MortarInfo& I = L.minfo[mi];
    if (I.q == 0) continue;
    I.geo = ng;
    ng += 8LL * (I.gmode ? (long long)I.q * I.q : 1);
    L.qmmax = std::max(L.qmmax, I.q);
    lists[size_t(I.em) * 6 + I.fm].push_back(int(mi) << 1);
    if (I.ep >= 0) lists[size_t(I.ep) * 6 + I.fp].push_back((int(mi) << 1) | 1);
  }
  L.mgeo.assign(size_t(ng), 0.0);
  parallel_for(M, [&](size_t mi) {
    const MortarInfo& I = L.minfo[mi];
    if (I.q == 0) return;
    const Mortar& mt = L.mortars[mi];
    const Cell& cm = L.cells[mt.em];
    const bool interior = mt.ep >= 0;
    const bool robin = !interior && mt.bc == 3;
    const int pm = pm_of[mi];
    const int q = I.q;
    double eta[kMaxQ + 1], wq[kMaxQ + 1];
    gauss_legendre(q, eta, wq);
    const int npts = I.gmode ? q * q : 1;
    double* out = L.mgeo.data() + I.geo;
    const int dmn = mt.fm >> 1;
    const double sgn = (mt.fm & 1) ? 1.0 : -1.0;
    for (int pidx = 0; pidx < npts; ++pidx) {
      const int c = pidx % q, d = pidx / q;
      const double s = I.gmode ? eta[c] : 0.0, t = I.gmode ? eta[d] : 0.0;
      double xim[3], x[3], J[3][3], Ji[3][3];
      face_ref(mt.fm, s, t, xim);
      cell_eval(mm, cm, xim, x, J);
      inv3(J, Ji);
      const double dj = det3(J);
      double nr = std::sqrt(Ji[dmn][0] * Ji[dmn][0] + Ji[dmn][1] * Ji[dmn][1] + Ji[dmn][2] * Ji[dmn][2]);
      double nh[3] = {sgn * Ji[dmn][0] / nr, sgn * Ji[dmn][1] / nr, sgn * Ji[dmn][2] / nr};
      const double S = dj * nr;
      double h = 2.0 / nr;
      double kx = kmt_of[mi], kxp = kpt_of[mi];
      if (I.gmode) side_k(mt, s, t, kx, kxp);
      double mminus[3], mplus[3] = {0, 0, 0};
      for (int r = 0; r < 3; ++r)
        mminus[r] = kx * (Ji[r][0] * nh[0] + Ji[r][1] * nh[1] + Ji[r][2] * nh[2]);
      if (interior) {
        double a, b, xip[3], xp[3], Jp[3][3], Jpi[3][3];
        plus_coords(mt.orient, mt.sub, s, t, a, b);
        face_ref(mt.fp, a, b, xip);
        cell_eval(mm, L.cells[mt.ep], xip, xp, Jp);
        inv3(Jp, Jpi);
        const int dp_ = mt.fp >> 1;
        const double nrp = std::sqrt(Jpi[dp_][0] * Jpi[dp_][0] + Jpi[dp_][1] * Jpi[dp_][1] +
                                     Jpi[dp_][2] * Jpi[dp_][2]);
        h = std::min(h, 2.0 / nrp);
        for (int r = 0; r < 3; ++r)
          mplus[r] = -kxp * (Jpi[r][0] * nh[0] + Jpi[r][1] * nh[1] + Jpi[r][2] * nh[2]);
      }
      double sigma = dp.C * pm * pm / h * std::max(kx, kxp);
      if (robin) {
        // Robin face: the only operator term is int gamma u v; with zero normal-derivative
        // coefficients the boundary flux w S (sigma u - n.grad u) of a Dirichlet face reduces to
        // w S gamma u (and its lift has no derivative part)
        for (int r = 0; r < 3; ++r) mminus[r] = 0.0;
        sigma = dp.robin_gamma;
      }
      const double wS = I.gmode ? wq[c] * wq[d] * S : S;
      double vals[8] = {mminus[0], mminus[1], mminus[2], mplus[0], mplus[1], mplus[2], wS, sigma};
      for (int k = 0; k < 8; ++k) out[size_t(k) * npts + pidx] = vals[k];
    }
  });
  L.fmlist.clear();
  for (size_t e = 0; e < E; ++e)
    for (int f = 0; f < 6; ++f) {
      auto& l = lists[e * 6 + f];
      L.einfo[e].fstart[f] = int(L.fmlist.size());
      L.einfo[e].fcnt[f] = int(l.size());
      L.fmlist.insert(L.fmlist.end(), l.begin(), l.end());
    }
  // ---- element-centric apply (fastapply.hip) ----
  // An element takes it when its map is affine and axis-aligned (constant diagonal metric, k
  // folded in), it has no mass term and p <= 7.  A face of such an element is evaluated there
  // (from both sides' coefficients) when it carries one mortar that is conforming (no sub-face)
  // with a constant metric whose normal coefficients have no tangential part, and the other
  // side is such an element too (or there is none: Dirichlet and Robin faces).  Every other
  // mortar stays with the mortar kernel, whose lifted terms (face slots) the element adds.
  L.fast.assign(E, 0);
  if (dp.ec_mode != 2) {
    long long nfast = 0;
    int nlo = kMaxN, nhi = 0;
    for (size_t e = 0; e < E; ++e) {
      const ElemInfo& I = L.einfo[e];
      if (I.vmode != 0 || I.mass || I.n < 2 || I.n > kFastMaxN) continue;
      const double* G = L.vgeo.data() + I.vgeo;
      if (G[1] != 0.0 || G[2] != 0.0 || G[4] != 0.0) continue;
      L.fast[e] = 1;
      nfast += 1;
      nlo = std::min(nlo, I.n);
      nhi = std::max(nhi, I.n);
    }
    // by level: from 4096 such elements up on levels of one degree and from 16384 up on levels
    // of several degrees (one launch per degree); below that the launches are latency bound and
    // the element and mortar kernels take less time
    if (dp.ec_mode == 0 && nfast < (nlo == nhi ? 4096 : 16384)) L.fast.assign(E, 0);
  }
  std::vector<unsigned char> mfast(M, 0);
  for (size_t mi = 0; mi < M; ++mi) {
    const MortarInfo& I = L.minfo[mi];
    if (I.q == 0 || I.gmode != 0 || I.sub >= 0 || !L.fast[I.em] || (I.ep >= 0 && !L.fast[I.ep])) continue;
    const double* g = L.mgeo.data() + I.geo;
    const int dm = I.fm >> 1;
    bool ok = true;
    for (int r = 0; r < 3; ++r) {
      if (r != dm && g[r] != 0.0) ok = false;
      if (I.ep >= 0 && r != (I.fp >> 1) && g[3 + r] != 0.0) ok = false;
    }
    mfast[mi] = ok ? 1 : 0;
  }
  L.flink.assign(E * 6, FaceLink{0, 0, 0});
  L.fcoef.clear();
  {
    std::map<std::array<double, 4>, int> coef_index;
    for (size_t e = 0; e < E; ++e) {
      if (!L.fast[e]) continue;
      const ElemInfo& I = L.einfo[e];
      for (int f = 0; f < 6; ++f) {
        FaceLink& fl = L.flink[e * 6 + f];
        if (I.fcnt[f] == 0) continue;  // kind 0
        const int ent = L.fmlist[size_t(I.fstart[f])];
        const int mi = ent >> 1, side = ent & 1;
        if (I.fcnt[f] != 1 || !mfast[size_t(mi)]) {
          fl.meta = 3;
          continue;
        }
        const MortarInfo& MI = L.minfo[size_t(mi)];
        const double* g = L.mgeo.data() + MI.geo;
        const bool interior = MI.ep >= 0;
        const int dm = MI.fm >> 1, dp_ = interior ? MI.fp >> 1 : 0;
        std::array<double, 4> c{g[6], g[7], 0.0, 0.0};
        if (side == 0) {
          c[2] = g[dm];
          c[3] = interior ? g[3 + dp_] : 0.0;
        } else {
          c[2] = g[3 + dp_];
          c[3] = g[dm];
        }
        auto it = coef_index.find(c);
        if (it == coef_index.end()) {
          it = coef_index.emplace(c, int(L.fcoef.size() / 4)).first;
          L.fcoef.insert(L.fcoef.end(), c.begin(), c.end());
        }
        fl.coef = it->second;
        if (!interior) {
          fl.meta = 2;
          continue;
        }
        // the neighbour's face coordinates of this face's nodes: (ia, ib) = swap ? (b, a) : (a, b),
        // then ia and ib reversed by flipA and flipB (the mortar's orientation seen from this side)
        const int o = MI.orient;
        int swp = o & 1, fa = (o >> 1) & 1, fb = (o >> 2) & 1;
        if (side == 1 && swp) std::swap(fa, fb);
        const int other = side == 0 ? MI.ep : MI.em;
        const int nf = side == 0 ? MI.fp : MI.fm;
        const ElemInfo& O = L.einfo[size_t(other)];
        // a neighbour of higher degree is read through the face trace it writes (value and
        // normal derivative at its face nodes, 2 nn^2 scalars) instead of its whole element
        fl.nb = O.n > I.n ? O.toff + 2LL * nf * O.n * O.n : O.off;
        fl.meta = 1 | (O.n << 2) | (nf << 7) | ((swp | (fa << 1) | (fb << 2)) << 10) | (O.n < I.n ? 1 << 13 : 0);
      }
    }
  }
  // buckets: fast elements by n (with the largest interior neighbour n), the others by (n, q)
  {
    L.fast_n.clear(); L.fast_nx.clear(); L.fast_start.clear(); L.fast_elems.clear();
    std::vector<std::pair<int, int>> kf;
    std::vector<std::pair<std::pair<int, int>, int>> keyed;
    for (size_t e = 0; e < E; ++e) {
      if (L.fast[e])
        kf.push_back({L.einfo[e].n, int(e)});
      else
        keyed.push_back({{L.einfo[e].n, L.einfo[e].q}, int(e)});
    }
    std::stable_sort(kf.begin(), kf.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t i = 0; i < kf.size(); ++i) {
      if (i == 0 || kf[i].first != kf[i - 1].first) {
        L.fast_n.push_back(kf[i].first);
        L.fast_nx.push_back(kf[i].first);
        L.fast_start.push_back((long long)i);
      }
      L.fast_elems.push_back(kf[i].second);
      for (int f = 0; f < 6; ++f) {
        const FaceLink& fl = L.flink[size_t(kf[i].second) * 6 + f];
        const int nn = (fl.meta >> 2) & 31;
        if ((fl.meta & 3) == 1 && nn != kf[i].first)  // a neighbour of another degree: mixed kernel
          L.fast_nx.back() = std::max(L.fast_nx.back(), std::max(nn, kf[i].first + 1));
      }
    }
    L.fast_start.push_back((long long)kf.size());
    // group order: face records, dof offsets and the diagonal metric of each fast element
    std::vector<FaceLink> byg(kf.size() * 6);
    L.fast_off.assign(kf.size(), 0);
    L.fast_toff.assign(kf.size(), 0);
    L.fast_g.assign(3 * kf.size(), 0.0);
    for (size_t i = 0; i < kf.size(); ++i) {
      const size_t e = size_t(kf[i].second);
      for (int f = 0; f < 6; ++f) byg[6 * i + f] = L.flink[6 * e + f];
      L.fast_off[i] = L.einfo[e].off;
      L.fast_toff[i] = L.einfo[e].toff;
      const double* G = L.vgeo.data() + L.einfo[e].vgeo;
      L.fast_g[3 * i] = G[0];
      L.fast_g[3 * i + 1] = G[3];
      L.fast_g[3 * i + 2] = G[5];
    }
    L.flink.swap(byg);
    std::stable_sort(keyed.begin(), keyed.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    L.bucket_n.clear(); L.bucket_q.clear(); L.bucket_start.clear(); L.bucket_elems.clear();
    for (size_t i = 0; i < keyed.size(); ++i) {
      if (i == 0 || keyed[i].first != keyed[i - 1].first) {
        L.bucket_n.push_back(keyed[i].first.first);
        L.bucket_q.push_back(keyed[i].first.second);
        L.bucket_start.push_back((long long)i);
      }
      L.bucket_elems.push_back(keyed[i].second);
    }
    L.bucket_start.push_back((long long)keyed.size());
  }
  // output slots of the mortar kernel: per element, 2 n^2 scalars per list entry in list order
  L.nslot = 0;
  for (size_t e = 0; e < E; ++e) {
    ElemInfo& I = L.einfo[e];
    I.soff = L.nslot;
    int cnt = 0;
    for (int f = 0; f < 6; ++f) cnt += I.fcnt[f];
    L.nslot += 2LL * cnt * I.n * I.n;
  }
  // one task per mortar that some face list holds (each side's list entry gives its slot)
  std::vector<long long> where(2 * L.minfo.size(), -1);
  for (size_t e = 0; e < E; ++e) {
    const ElemInfo& I = L.einfo[e];
    for (int f = 0; f < 6; ++f)
      for (int r = 0; r < I.fcnt[f]; ++r) {
        const int k = I.fstart[f] + r;
        where[size_t(L.fmlist[k])] = I.soff + 2LL * (k - I.fstart[0]) * I.n * I.n;
      }
  }
  L.mtask.clear();
  std::vector<unsigned char> traced(E, 0);
  for (size_t m = 0; m < L.minfo.size(); ++m) {
    if (where[2 * m] < 0 && where[2 * m + 1] < 0) continue;
    if (mfast[m]) continue;  // evaluated by the element-centric apply on both sides
    const MortarInfo& M = L.minfo[m];
    if (where[2 * m] < 0 || (M.ep >= 0) != (where[2 * m + 1] >= 0))
      throw Error(-2, "internal: a mortar listed on one side of an interior face only");
    MortarTask t = mortar_task(L, M);
    for (int sd = 0; sd < 1 + t.interior; ++sd) {
      t.slot[sd] = where[2 * m + sd];
      traced[size_t(sd ? M.ep : M.em)] = 1;
    }
    L.mtask.push_back(t);
  }
  L.trace_elems.clear();
  for (size_t e = 0; e < E; ++e)
    if (traced[e]) L.trace_elems.push_back(int(e));
  (void)T;
}

void build_transfer(LevelHost& fine, const LevelHost& coarse) {
  std::vector<int> parent, bits;
  parent_cells(fine.cells, coarse.cells, parent, bits);
  const size_t E = fine.cells.size();
  fine.tinfo.resize(E);
  std::vector<int> cnt(coarse.cells.size() + 1, 0);
  for (size_t e = 0; e < E; ++e) {
    TransferInfo& t = fine.tinfo[e];
    t.foff = fine.einfo[e].off;
    t.coff = coarse.einfo[parent[e]].off;
    t.nf = fine.einfo[e].n;
    t.nc = coarse.einfo[parent[e]].n;
    t.bits = bits[e];
    t.pad = 0;
    if (t.nc > t.nf) throw Error(-2, "coarse degree above the fine degree");
    cnt[parent[e] + 1]++;
  }
  fine.cstart.assign(coarse.cells.size() + 1, 0);
  for (size_t K = 0; K < coarse.cells.size(); ++K) fine.cstart[K + 1] = fine.cstart[K] + cnt[K + 1];
  fine.clist.assign(E, 0);
  std::vector<int> fill(fine.cstart.begin(), fine.cstart.end() - 1);
  for (size_t e = 0; e < E; ++e) fine.clist[fill[parent[e]]++] = int(e);
}

// ---------------------------------------------------------------------------------
void build_diagonal(const OpTable& T, LevelHost& L) {
  L.diag.assign(size_t(L.ndof), 0.0);
  const double* td = T.data.data();
  // one element per task: its volume part, then its sides of its mortars in mortar order (each
  // entry sums its terms in the same order whatever the number of threads)
  parallel_for(L.einfo.size(), [&](size_t e) {
    const ElemInfo& I = L.einfo[e];
    std::vector<double> t1, t2;
    {
      const int n = I.n, q = I.q, q3 = q * q * q;
      const double* B = td + T.index(OpTable::GL_VAL, n, q);
      const double* Dt = td + T.index(OpTable::GL_DER, n, q);
      const double* w = td + T.w_off[q];
      const double* G = L.vgeo.data() + I.vgeo;
      double* out = L.diag.data() + I.off;
      const double* fac[2] = {B, Dt};
      const int pr[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
      t1.assign(size_t(q) * q * n, 0.0);
      t2.assign(size_t(q) * n * n, 0.0);
      for (int m = 0; m < 6; ++m) {
        const int d0 = pr[m][0], d1 = pr[m][1];
        const double mult = d0 == d1 ? 1.0 : 2.0;
        // factor along axis x of phi_d phi_d' : derivative where the axis is d or d'
        const double* X0 = fac[d0 == 0]; const double* X1 = fac[d1 == 0];
        const double* Y0 = fac[d0 == 1]; const double* Y1 = fac[d1 == 1];
        const double* Z0 = fac[d0 == 2]; const double* Z1 = fac[d1 == 2];
        auto g = [&](int idx) {
          if (I.vmode == 0) {
            const int a = idx % q, b = (idx / q) % q, c = idx / (q * q);
            return G[m] * w[a] * w[b] * w[c];
          }
          return G[size_t(m) * q3 + idx];
        };
        // t1[c][b][i] = sum_a X0[a][i] X1[a][i] g[c][b][a]
        for (int cb = 0; cb < q * q; ++cb)
          for (int i = 0; i < n; ++i) {
            double s = 0;
            for (int a = 0; a < q; ++a) s += X0[a * n + i] * X1[a * n + i] * g(cb * q + a);
            t1[size_t(cb) * n + i] = s;
          }
        // t2[c][j][i] = sum_b Y0[b][j] Y1[b][j] t1[c][b][i]
        for (int c = 0; c < q; ++c)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              double s = 0;
              for (int b = 0; b < q; ++b) s += Y0[b * n + j] * Y1[b * n + j] * t1[(size_t(c) * q + b) * n + i];
              t2[(size_t(c) * n + j) * n + i] = s;
            }
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              double s = 0;
              for (int c = 0; c < q; ++c) s += Z0[c * n + k] * Z1[c * n + k] * t2[(size_t(c) * n + j) * n + i];
              out[(k * n + j) * n + i] += mult * s;
            }
      }
    }
    // faces: psi^2 sigma and the consistency/symmetry self terms, face nodes only
    std::vector<int> ents;
    for (int f = 0; f < 6; ++f)
      for (int r = 0; r < I.fcnt[f]; ++r) ents.push_back(L.fmlist[size_t(I.fstart[f] + r)]);
    std::sort(ents.begin(), ents.end());
    for (int ent : ents) {
      const MortarInfo& M = L.minfo[size_t(ent >> 1)];
      const int side = ent & 1;
      if (M.q == 0) continue;
      const int q = M.q;
      const bool interior = M.ep >= 0;
      const double factor = interior ? 1.0 : 2.0;
      const double* wq = td + T.w_off[q];
      const double* mg = L.mgeo.data() + M.geo;
      const int npts = M.gmode ? q * q : 1;
      const int f = side ? M.fp : M.fm;
      const int n = I.n, d = f >> 1, t0 = d == 0 ? 1 : 0, t1_ = d == 2 ? 1 : 2;
      const SideMap sm = side_map(M, side);
      const double* La = td + T.index(OpTable::GL_VAL + 2 * sm.halfA, n, q);
      const double* Da = td + T.index(OpTable::GL_DER + 2 * sm.halfA, n, q);
      const double* Lb = td + T.index(OpTable::GL_VAL + 2 * sm.halfB, n, q);
      const double* Db = td + T.index(OpTable::GL_DER + 2 * sm.halfB, n, q);
      const double* dface = td + T.dface_off[n] + ((f & 1) ? n : 0);
      const int kf = (f & 1) ? n - 1 : 0;
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double s = 0;
          for (int y = 0; y < q; ++y)
            for (int x = 0; x < q; ++x) {
              const int c = sm.swap ? y : x, dd = sm.swap ? x : y;
              const int rho = c + q * dd;
              const int ra = sm.flipA ? q - 1 - x : x, rb = sm.flipB ? q - 1 - y : y;
              const int p = M.gmode ? rho : 0;
              const double wS = M.gmode ? mg[6 * npts + p] : wq[c] * wq[dd] * mg[6];
              const double sig = mg[7 * npts + p];
              const double ma = mg[(3 * side + t0) * npts + p];
              const double mb = mg[(3 * side + t1_) * npts + p];
              const double mn = mg[(3 * side + d) * npts + p];
              const double la = La[ra * n + i], lb = Lb[rb * n + j];
              const double psi = la * lb;
              const double gn = ma * Da[ra * n + i] * lb + mb * la * Db[rb * n + j] + mn * psi * dface[kf];
              s += wS * (sig * psi * psi - factor * psi * gn);
            }
          int idx[3];
          idx[d] = kf; idx[t0] = i; idx[t1_] = j;
          L.diag[size_t(I.off) + (idx[2] * n + idx[1]) * n + idx[0]] += s;
        }
    }
  });
}

// ---------------------------------------------------------------------------------
namespace {

// constant-density star (Sec. III.B): C = (2 pi rho0 / 3)^(-1/4); alpha from the continuity
// of psi and dpsi/dr at r0, rho0 r0^2 = (3 / (2 pi)) alpha^10 / (1 + alpha^2)^6, on the
// weak-field branch alpha >= sqrt(5) (bisection; the right side falls there);
// beta = r0 (C u_alpha(r0) - 1); psi = C u_alpha(r) inside r0, beta / r + 1 outside
double star_psi(double rho0, double r0, double r) {
  const double C = std::pow(2.0 * M_PI * rho0 / 3.0, -0.25);
  const double target = rho0 * r0 * r0;
  auto f = [&](double a) { return 3.0 / (2.0 * M_PI) * std::pow(a, 10) / std::pow(1.0 + a * a, 6) - target; };
  double lo = std::sqrt(5.0), hi = 2.0 * lo;
  if (f(lo) < 0) return std::nan("");
  while (f(hi) > 0) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    (f(mid) > 0 ? lo : hi) = mid;
  }
  const double alpha = 0.5 * (lo + hi), ar = alpha * r0;
  if (r <= r0) return C * std::sqrt(ar) / std::sqrt(r * r + ar * ar);
  const double beta = r0 * (C * std::sqrt(ar) / std::sqrt(r0 * r0 + ar * ar) - 1.0);
  return beta / r + 1.0;
}

double exact_u(int kind, const std::vector<double>& P, const double x[3]) {
  const double X = x[0], Y = x[1], Z = x[2];
  switch (kind) {
    case 0: return std::sin(M_PI * X) * std::sin(M_PI * Y) * std::sin(M_PI * Z);
    case 1: {
      const double r = std::sqrt(X * X + Y * Y + Z * Z);
      return 1.0 / r + P[0] * X * Z / (r * r * r * r * r);
    }
    case 2: {
      const double r2 = X * X + Y * Y + Z * Z;
      if (std::sqrt(r2) < P[0]) return r2 / P[1] + P[0] * P[0] * (1.0 / P[2] - 1.0 / P[1]);
      return r2 / P[2];
    }
    case 3:
    case 5: {  // polynomial (5: Dirichlet data only, no source)
      const int K = int(std::lround(std::cbrt(double(P.size()))));
      double u = 0;
      for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b)
          for (int c = 0; c < K; ++c)
            u += P[(a * K + b) * K + c] * std::pow(X, a) * std::pow(Y, b) * std::pow(Z, c);
      return u;
    }
    case 6: return star_psi(P[0], P[1], std::sqrt(X * X + Y * Y + Z * Z));
    default: return 0.0;
  }
}

// grad u of the manufactured u for the kinds with Neumann data (sin sin sin, the polynomial
// kinds); false for the others
bool exact_grad(int kind, const std::vector<double>& P, const double x[3], double g[3]) {
  const double X = x[0], Y = x[1], Z = x[2];
  if (kind == 0) {
    const double sx = std::sin(M_PI * X), sy = std::sin(M_PI * Y), sz = std::sin(M_PI * Z);
    g[0] = M_PI * std::cos(M_PI * X) * sy * sz;
    g[1] = M_PI * sx * std::cos(M_PI * Y) * sz;
    g[2] = M_PI * sx * sy * std::cos(M_PI * Z);
    return true;
  }
  if (kind == 3 || kind == 5) {
    const int K = int(std::lround(std::cbrt(double(P.size()))));
    g[0] = g[1] = g[2] = 0;
    for (int a = 0; a < K; ++a)
      for (int b = 0; b < K; ++b)
        for (int c = 0; c < K; ++c) {
          const double C = P[(a * K + b) * K + c];
          if (a >= 1) g[0] += C * a * std::pow(X, a - 1) * std::pow(Y, b) * std::pow(Z, c);
          if (b >= 1) g[1] += C * b * std::pow(X, a) * std::pow(Y, b - 1) * std::pow(Z, c);
          if (c >= 1) g[2] += C * c * std::pow(X, a) * std::pow(Y, b) * std::pow(Z, c - 1);
        }
    return true;
  }
  return false;
}

double source(int kind, const std::vector<double>& P, const double x[3]) {
  return rhs_source(kind, P.data(), int(P.size()), x);
}

}  // namespace

void nl_coefficients(int kind, const std::vector<double>& P, const double x[3], double& alpha, double& beta) {
  const double X = x[0], Y = x[1], Z = x[2];
  if (kind == 0) {  // puncture: P = [s, rows (cx, cy, cz, m, a)]
    const double s = P[0];
    double psum = 0, b = 0;
    for (size_t r = 1; r + 4 < P.size(); r += 5) {
      const double dx = X - P[r], dy = Y - P[r + 1], dz = Z - P[r + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      psum += P[r + 3] / (2.0 * std::sqrt(r2));
      b += P[r + 4] * std::exp(-r2 / (2.0 * s * s));
    }
    const double q = 1.0 + X * X + Y * Y + Z * Z;
    alpha = 1.0 / (1.0 + psum);
    beta = b / (q * q);
  } else if (kind == 2) {  // constant-density star: P = [rho0, r0], beta = 2 pi rho (alpha unused)
    alpha = 0.0;
    beta = std::sqrt(X * X + Y * Y + Z * Z) <= P[1] ? 2.0 * M_PI * P[0] : 0.0;
  } else {  // quadratic manufactured: P = [alpha, C (27)], beta = (-lap u*) (1 + alpha u*)^7
    alpha = P[0];
    const std::vector<double> C(P.begin() + 1, P.end());
    const double u = exact_u(3, C, x), g = source(3, C, x), s = 1.0 + alpha * u;
    const double s2 = s * s, s4 = s2 * s2;
    beta = g * s4 * s2 * s;
  }
}

void mass_points(const MacroMesh& mm, const LevelHost& L, std::vector<double>& x, std::vector<double>& wdet) {
  x.assign(3 * size_t(L.nmq), 0.0);
  wdet.assign(size_t(L.nmq), 0.0);
  double eta[kMaxQ + 1], wq[kMaxQ + 1];
  for (size_t e = 0; e < L.cells.size(); ++e) {
    const ElemInfo& I = L.einfo[e];
    if (!I.mass) continue;
    const int q = I.q;
    gauss_legendre(q, eta, wq);
    for (int c = 0; c < q; ++c)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          const double xi[3] = {eta[a], eta[b], eta[c]};
          double xp[3], J[3][3];
          cell_eval(mm, L.cells[e], xi, xp, J);
          const size_t k = size_t(I.mq) + a + size_t(q) * (b + size_t(q) * c);
          for (int d = 0; d < 3; ++d) x[3 * k + d] = xp[d];
          wdet[k] = wq[a] * wq[b] * wq[c] * det3(J);
        }
  }
}

void mass_table(const MacroMesh& mm, const DiscParams& dp, const LevelHost& L, std::vector<double>& wc) {
  wc.assign(size_t(L.nmq), 0.0);
  double eta[kMaxQ + 1], wq[kMaxQ + 1];
  for (size_t e = 0; e < L.cells.size(); ++e) {
    const ElemInfo& I = L.einfo[e];
    if (!I.mass) continue;
    const int q = I.q;
    gauss_legendre(q, eta, wq);
    for (int c = 0; c < q; ++c)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          const double xi[3] = {eta[a], eta[b], eta[c]};
          double xp[3], J[3][3];
          cell_eval(mm, L.cells[e], xi, xp, J);
          const size_t k = size_t(I.mq) + a + size_t(q) * (b + size_t(q) * c);
          wc[k] = wq[a] * wq[b] * wq[c] * det3(J) * field_point(dp.cfield, L.cvals, L, int(e), xi);
        }
  }
}

void assemble_rhs(const MacroMesh& mm, const DiscParams& dp, const OpTable& T, const LevelHost& L,
                  int kind, const std::vector<double>& P, std::vector<double>& F) {
  F.assign(size_t(L.ndof), 0.0);
  const double* td = T.data.data();
  // volume terms int g psi: on the device (rhs.hip), added to these face terms
  // Dirichlet faces: int g_D (sigma psi - k n.grad psi), with the face's own rule (a flat face
  // whose rule was raised to the volume rule's keeps its constant metric, valid at any q)
  for (size_t mi = 0; mi < L.minfo.size(); ++mi) {
    const MortarInfo& M = L.minfo[mi];
    if (M.q == 0 || M.ep >= 0 || M.bc == 3) continue;
    const int q = M.rq;
    const ElemInfo& I = L.einfo[M.em];
    const int n = I.n, f = M.fm, d = f >> 1, t0 = d == 0 ? 1 : 0, t1_ = d == 2 ? 1 : 2;
    const double* La = td + T.index(OpTable::GL_VAL, n, q);
    const double* Da = td + T.index(OpTable::GL_DER, n, q);
    const double* wq = td + T.w_off[q];
    const double* eta = td + T.gl_off[q];
    const double* dface = td + T.dface_off[n] + ((f & 1) ? n : 0);
    const double* mg = L.mgeo.data() + M.geo;
    const int npts = M.gmode ? q * q : 1;
    const int kf = (f & 1) ? n - 1 : 0;
    for (int y = 0; y < q; ++y)
      for (int x = 0; x < q; ++x) {
        const int rho = x + q * y, p = M.gmode ? rho : 0;
        double xi[3], xx[3], J[3][3];
        xi[d] = (f & 1) ? 1.0 : -1.0;
        xi[t0] = eta[x];
        xi[t1_] = eta[y];
        cell_eval(mm, L.cells[M.em], xi, xx, J);
        const double gd = exact_u(kind, P, xx);
        const double wS = M.gmode ? mg[6 * npts + p] : wq[x] * wq[y] * mg[6];
        const double A = wS * mg[7 * npts + p] * gd;
        const double Bc = -wS * gd;
        const double ma = mg[t0 * npts + p], mb = mg[t1_ * npts + p], mn = mg[d * npts + p];
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            const double la = La[x * n + i], lb = La[y * n + j];
            const double face = A * la * lb + Bc * (ma * Da[x * n + i] * lb + mb * la * Da[y * n + j]);
            int idx[3];
            idx[t0] = i; idx[t1_] = j;
            for (int k = 0; k < n; ++k) {
              idx[d] = k;
              double v = Bc * mn * la * lb * dface[k];
              if (k == kf) v += face;
              F[size_t(I.off) + (idx[2] * n + idx[1]) * n + idx[0]] += v;
            }
          }
      }
  }
  // Neumann faces (Eq. NeumannBC): int g_N psi, g_N = k grad u . n (outward n; 0 for the
  // Gaussian sources), with the face's own rule (n points, n + quad_extra on curved faces or
  // with variable k); only the face layer of the element's nodes is nonzero on the face.
  // Robin faces (Eq. RobinBC, read with the sign of Eq. lh): int g_R psi with
  // g_R = k n.grad u + gamma u (the gamma u v part is in the operator)
  for (size_t mi = 0; mi < L.minfo.size(); ++mi) {
    const MortarInfo& M = L.minfo[mi];
    if (M.ep >= 0 || (M.bc != 2 && M.bc != 3)) continue;
    if (kind != 4) {
      double g0[3];
      const double x0[3] = {0, 0, 0};
      if (!exact_grad(kind, P, x0, g0)) throw Error(-7, "no Neumann data for this right-hand-side kind");
    }
    const ElemInfo& I = L.einfo[M.em];
    const Cell& cell = L.cells[M.em];
    const bool curved = mm.macros[cell.macro].kind != 0;
    const int n = I.n, q = n + ((curved || !kconst(dp)) ? dp.quad_extra : 0);
    if (q > kMaxQ) throw Error(-2, "too many quadrature points");
    const int f = M.fm, d = f >> 1, t0 = d == 0 ? 1 : 0, t1_ = d == 2 ? 1 : 2;
    const double sgn = (f & 1) ? 1.0 : -1.0;
    const double* La = td + T.index(OpTable::GL_VAL, n, q);
    const double* wq = td + T.w_off[q];
    const double* eta = td + T.gl_off[q];
    const int kf = (f & 1) ? n - 1 : 0;
    for (int y = 0; y < q; ++y)
      for (int x = 0; x < q; ++x) {
        double xi[3], xx[3], J[3][3], Ji[3][3], g[3] = {0, 0, 0};
        xi[d] = sgn;
        xi[t0] = eta[x];
        xi[t1_] = eta[y];
        cell_eval(mm, cell, xi, xx, J);
        inv3(J, Ji);
        const double nr = std::sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
        if (kind != 4) exact_grad(kind, P, xx, g);
        double gN = k_point(dp, L, M.em, xi, xx) * sgn * (Ji[d][0] * g[0] + Ji[d][1] * g[1] + Ji[d][2] * g[2]) / nr;
        if (M.bc == 3 && kind != 4) gN += dp.robin_gamma * exact_u(kind, P, xx);
        const double v = wq[x] * wq[y] * det3(J) * nr * gN;
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            int idx[3];
            idx[d] = kf;
            idx[t0] = i;
            idx[t1_] = j;
            F[size_t(I.off) + (idx[2] * n + idx[1]) * n + idx[0]] += v * La[x * n + i] * La[y * n + j];
          }
      }
  }
}

// ---- a posteriori estimator: point data (Eqs. Eta2_Integrals) -----------------------------
void estimator_tables(const MacroMesh& mm, const MacroMesh* grid, const DiscParams& dp, const LevelHost& L,
                      int kind, const std::vector<double>& P, EstTables& out) {
  (void)dp;
  const MacroMesh& gm = grid ? *grid : mm;
  const size_t E = L.cells.size();
  out = EstTables{};
  out.voff.resize(E);
  out.he2p2.resize(E);
  long long nv = 0;
  for (size_t e = 0; e < E; ++e) {
    out.voff[e] = nv;
    nv += 3LL * L.einfo[e].q * L.einfo[e].q * L.einfo[e].q;
  }
  out.vol.assign(size_t(nv), 0.0);
  parallel_for(E, [&](size_t e) {
    const ElemInfo& I = L.einfo[e];
    const Cell& c = L.cells[e];
    const int q = I.q;
    double eta[kMaxQ + 1], wq[kMaxQ + 1];
    gauss_legendre(q, eta, wq);
    double* o = out.vol.data() + out.voff[e];
    for (int cc = 0; cc < q; ++cc)
      for (int b = 0; b < q; ++b)
        for (int a = 0; a < q; ++a) {
          double xi[3] = {eta[a], eta[b], eta[cc]}, x[3], J[3][3], xg[3], Jg[3][3];
          cell_eval(mm, c, xi, x, J);
          const double dj = det3(J);
          double djg = dj;
          if (grid) {
            cell_eval(gm, c, xi, xg, Jg);
            djg = det3(Jg);
            if (!(djg > 0)) throw Error(-2, "estimator grid: non-positive Jacobian determinant");
          }
          const size_t k = 3 * size_t(a + q * (b + q * cc));
          o[k] = wq[a] * wq[b] * wq[cc] * djg;
          o[k + 1] = 1.0 / dj;
          o[k + 2] = source(kind, P, x);
        }
    // h_e: the largest distance between two of the element's vertices
    double X[8][3];
    for (int v = 0; v < 8; ++v) {
      double xi[3] = {(v & 1) ? 1.0 : -1.0, (v & 2) ? 1.0 : -1.0, (v & 4) ? 1.0 : -1.0}, J[3][3];
      cell_eval(gm, c, xi, X[v], J);
    }
    double h2 = 0;
    for (int v = 0; v < 8; ++v)
      for (int w = v + 1; w < 8; ++w) {
        const double dx = X[v][0] - X[w][0], dy = X[v][1] - X[w][1], dz = X[v][2] - X[w][2];
        h2 = std::max(h2, dx * dx + dy * dy + dz * dz);
      }
    out.he2p2[e] = h2 * double(c.p) * double(c.p);
  });
  // at reference point xi of cell c: S = det J |grad xi_d| and 2 / |grad xi_d| on mesh m
  auto face_metric = [](const MacroMesh& m, const Cell& c, const double xi[3], int d, double& S, double& h,
                        double x[3]) {
    double J[3][3], Ji[3][3];
    cell_eval(m, c, xi, x, J);
    inv3(J, Ji);
    const double nr = std::sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
    S = det3(J) * nr;
    h = 2.0 / nr;
  };
  long long nf = 0;
  for (size_t m = 0; m < L.minfo.size(); ++m) {
    const MortarInfo& M = L.minfo[m];
    if (M.q == 0 || (M.ep < 0 && M.bc != 1)) continue;  // Neumann, Robin: no estimator term
    out.tasks.push_back(mortar_task(L, M));
    out.task_mortar.push_back(int(m));
    out.foff.push_back(nf);
    nf += 4LL * M.q * M.q;
  }
  out.face.assign(size_t(nf), 0.0);
  parallel_for(out.tasks.size(), [&](size_t t) {
    const MortarInfo& M = L.minfo[size_t(out.task_mortar[t])];
    const int q = M.q;
    double eta[kMaxQ + 1], wq[kMaxQ + 1];
    gauss_legendre(q, eta, wq);
    const Cell& cm = L.cells[M.em];
    const int pm = std::max(cm.p, M.ep >= 0 ? L.cells[M.ep].p : 0);
    double* o = out.face.data() + out.foff[t];
    for (int d = 0; d < q; ++d)
      for (int ci = 0; ci < q; ++ci) {
        double xim[3], x[3], xg[3], S, h, Sg, hg;
        face_ref(M.fm, eta[ci], eta[d], xim);
        face_metric(mm, cm, xim, M.fm >> 1, S, h, x);
        Sg = S;
        hg = h;
        if (grid) face_metric(gm, cm, xim, M.fm >> 1, Sg, hg, xg);
        if (M.ep >= 0) {
          double a, b, xip[3], xp[3], Sp, hp;
          plus_coords(M.orient, M.sub, eta[ci], eta[d], a, b);
          face_ref(M.fp, a, b, xip);
          face_metric(mm, L.cells[M.ep], xip, M.fp >> 1, Sp, hp, xp);
          h = std::min(h, hp);
          if (grid) {
            face_metric(gm, L.cells[M.ep], xip, M.fp >> 1, Sp, hp, xp);
            hg = std::min(hg, hp);
          } else {
            hg = h;
          }
        }
        if (!(Sg > 0)) throw Error(-2, "estimator grid: non-positive face Jacobian");
        const size_t k = 4 * size_t(ci + q * d);
        o[k] = hg / double(pm);
        o[k + 1] = M.ep >= 0 ? 0.0 : exact_u(kind, P, x);
        o[k + 2] = Sg / S;
        o[k + 3] = h / hg;
      }
  });
}

}  // namespace hpdg
