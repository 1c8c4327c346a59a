// Octree-forest topology: mortar elements of a 2:1-balanced mesh (Sec. II.A.1) and the
// multigrid mesh hierarchy (Sec. II.D.3: naive coarsening of complete sibling families,
// refinement where the result violates 2:1 face balance, coarse degree = min of the
// children, cells that are not coarsened keep their degree).
#include <algorithm>
#include <unordered_map>

#include "host.hpp"

namespace hpdg {

namespace {

inline uint64_t key_of(int m, int l, int a0, int a1, int a2) {
  return (uint64_t(m) << 47) | (uint64_t(l) << 42) | (uint64_t(a0) << 28) | (uint64_t(a1) << 14) |
         uint64_t(a2);
}

inline void tangential(int d, int& t0, int& t1) {
  t0 = d == 0 ? 1 : 0;
  t1 = d == 2 ? 1 : 2;
}

// The cell of the same level across face f of (m, l, a): returns false on the boundary.
bool across(const MacroMesh& mm, int m, int l, const int a[3], int f, int& mb, int b[3], int& fb,
            int& o) {
  const int d = f >> 1, s = f & 1, n = 1 << l;
  b[0] = a[0];
  b[1] = a[1];
  b[2] = a[2];
  b[d] += s ? 1 : -1;
  if (b[d] >= 0 && b[d] < n) {
    mb = m;
    fb = f ^ 1;
    o = 0;
    return true;
  }
  mb = mm.nbr[6 * m + f];
  if (mb < 0) return false;
  fb = mm.nbr_face[6 * m + f];
  o = mm.nbr_orient[6 * m + f];
  int t0, t1, u0, u1;
  tangential(d, t0, t1);
  tangential(fb >> 1, u0, u1);
  int ca = (o & 1) ? a[t1] : a[t0];
  int cb = (o & 1) ? a[t0] : a[t1];
  if (o & 2) ca = n - 1 - ca;
  if (o & 4) cb = n - 1 - cb;
  b[fb >> 1] = (fb & 1) ? n - 1 : 0;
  b[u0] = ca;
  b[u1] = cb;
  return true;
}

// 2:1 restoration: a leaf adjacent to a leaf two or more levels finer is refined (its
// children keep its degree), until no such pair is left
void balance_leaves(const MacroMesh& mm, std::unordered_map<uint64_t, Cell>& leaves) {
  auto covering = [&](int m, int l, const int a[3]) -> Cell* {
    for (int lev = l; lev >= 0; --lev) {
      int sh = l - lev;
      auto it = leaves.find(key_of(m, lev, a[0] >> sh, a[1] >> sh, a[2] >> sh));
      if (it != leaves.end()) return &it->second;
    }
    return nullptr;
  };
  bool changed = true;
  while (changed) {
    changed = false;
    std::vector<Cell> snapshot;
    snapshot.reserve(leaves.size());
    for (auto& kv : leaves) snapshot.push_back(kv.second);
    std::sort(snapshot.begin(), snapshot.end(), [](const Cell& x, const Cell& y) {
      if (x.level != y.level) return x.level > y.level;
      if (x.macro != y.macro) return x.macro < y.macro;
      for (int d = 0; d < 3; ++d)
        if (x.a[d] != y.a[d]) return x.a[d] < y.a[d];
      return false;
    });
    for (const Cell& c : snapshot) {
      if (!leaves.count(key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2]))) continue;
      for (int f = 0; f < 6; ++f) {
        int mb, b[3], fb, o;
        if (!across(mm, c.macro, c.level, c.a, f, mb, b, fb, o)) continue;
        Cell* lf = covering(mb, c.level, b);
        if (lf && lf->level <= c.level - 2) {
          Cell par = *lf;
          leaves.erase(key_of(par.macro, par.level, par.a[0], par.a[1], par.a[2]));
          for (int z = 0; z < 8; ++z) {
            Cell k{par.macro, par.level + 1,
                   {2 * par.a[0] + (z & 1), 2 * par.a[1] + ((z >> 1) & 1), 2 * par.a[2] + (z >> 2)},
                   par.p};
            leaves[key_of(k.macro, k.level, k.a[0], k.a[1], k.a[2])] = k;
          }
          changed = true;
        }
      }
    }
  }
}

}  // namespace

std::vector<Mortar> find_mortars(const MacroMesh& mm, const std::vector<Cell>& cells) {
  std::unordered_map<uint64_t, int> idx;
  idx.reserve(cells.size() * 2);
  for (size_t e = 0; e < cells.size(); ++e) {
    const Cell& c = cells[e];
    if (c.level > 14 || c.macro < 0 || c.macro >= int(mm.macros.size()))
      throw Error(-2, "cell outside the macro-mesh");
    for (int d = 0; d < 3; ++d)
      if (c.a[d] < 0 || c.a[d] >= (1 << c.level)) throw Error(-2, "anchor outside its macro");
    if (!idx.emplace(key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2]), int(e)).second)
      throw Error(-2, "duplicate cell");
  }
  std::vector<Mortar> out;
  for (size_t e = 0; e < cells.size(); ++e) {
    const Cell& c = cells[e];
    for (int f = 0; f < 6; ++f) {
      int mb, b[3], fb, o;
      if (!across(mm, c.macro, c.level, c.a, f, mb, b, fb, o)) {
        out.push_back({int(e), f, -1, -1, 0, -1, mm.bc[6 * c.macro + f]});
        continue;
      }
      auto it = idx.find(key_of(mb, c.level, b[0], b[1], b[2]));
      if (it != idx.end()) {
        if (int(e) < it->second) out.push_back({int(e), f, it->second, fb, o, -1, 0});
        continue;
      }
      if (c.level > 0) {
        it = idx.find(key_of(mb, c.level - 1, b[0] >> 1, b[1] >> 1, b[2] >> 1));
        if (it != idx.end()) {
          int u0, u1;
          tangential(fb >> 1, u0, u1);
          out.push_back({int(e), f, it->second, fb, o, (b[u0] & 1) + 2 * (b[u1] & 1), 0});
          continue;
        }
      }
      // the neighbour is refined: its four children on this face must exist
      const int db = fb >> 1, side = fb & 1;
      int kids = 0;
      for (int z = 0; z < 8; ++z) {
        int bits[3] = {z & 1, (z >> 1) & 1, (z >> 2) & 1};
        if (bits[db] != side) continue;
        if (idx.count(key_of(mb, c.level + 1, 2 * b[0] + bits[0], 2 * b[1] + bits[1],
                             2 * b[2] + bits[2])))
          ++kids;
      }
      if (kids != 4) throw Error(-2, "mesh is not 2:1 balanced (or a face is unmatched)");
    }
  }
  return out;
}

bool coarsen_cells(const MacroMesh& mm, const std::vector<Cell>& fine, std::vector<Cell>& coarse) {
  // complete sibling families -> parent with the minimum degree
  std::unordered_map<uint64_t, std::vector<int>> fam;
  for (size_t e = 0; e < fine.size(); ++e) {
    const Cell& c = fine[e];
    if (c.level == 0) continue;
    fam[key_of(c.macro, c.level - 1, c.a[0] >> 1, c.a[1] >> 1, c.a[2] >> 1)].push_back(int(e));
  }
  std::unordered_map<uint64_t, Cell> leaves;
  std::vector<char> merged(fine.size(), 0);
  for (auto& kv : fam) {
    if (kv.second.size() != 8) continue;
    const Cell& c0 = fine[kv.second[0]];
    Cell p{c0.macro, c0.level - 1, {c0.a[0] >> 1, c0.a[1] >> 1, c0.a[2] >> 1}, 1 << 30};
    for (int e : kv.second) {
      p.p = std::min(p.p, fine[e].p);
      merged[e] = 1;
    }
    leaves[kv.first] = p;
  }
  if (leaves.empty()) return false;
  for (size_t e = 0; e < fine.size(); ++e)
    if (!merged[e]) {
      const Cell& c = fine[e];
      leaves[key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2])] = c;
    }
  balance_leaves(mm, leaves);
  if (leaves.size() == fine.size()) {
    bool same = true;
    for (const Cell& c : fine)
      if (!leaves.count(key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2]))) same = false;
    if (same) return false;
  }
  coarse.clear();
  for (auto& kv : leaves) coarse.push_back(kv.second);
  std::sort(coarse.begin(), coarse.end(), [](const Cell& x, const Cell& y) {
    if (x.p != y.p) return x.p < y.p;
    if (x.macro != y.macro) return x.macro < y.macro;
    if (x.level != y.level) return x.level < y.level;
    for (int d = 2; d >= 0; --d)
      if (x.a[d] != y.a[d]) return x.a[d] < y.a[d];
    return false;
  });
  return true;
}

void parent_cells(const std::vector<Cell>& fine, const std::vector<Cell>& coarse,
                  std::vector<int>& parent, std::vector<int>& bits) {
  std::unordered_map<uint64_t, int> idx;
  for (size_t e = 0; e < coarse.size(); ++e) {
    const Cell& c = coarse[e];
    idx[key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2])] = int(e);
  }
  parent.resize(fine.size());
  bits.resize(fine.size());
  for (size_t e = 0; e < fine.size(); ++e) {
    const Cell& c = fine[e];
    auto it = idx.find(key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2]));
    if (it != idx.end()) {
      parent[e] = it->second;
      bits[e] = -1;
      continue;
    }
    it = idx.find(key_of(c.macro, c.level - 1, c.a[0] >> 1, c.a[1] >> 1, c.a[2] >> 1));
    if (it == idx.end()) throw Error(-2, "multigrid hierarchy: fine cell without a coarse cell");
    parent[e] = it->second;
    bits[e] = (c.a[0] & 1) | ((c.a[1] & 1) << 1) | ((c.a[2] & 1) << 2);
  }
}

void adapt_cells(const MacroMesh& mm, const std::vector<Cell>& cells, const signed char* action, int max_p,
                 std::vector<Cell>& out, std::vector<int>& origin) {
  (void)find_mortars(mm, cells);  // the input must be a valid 2:1-balanced mesh
  std::unordered_map<uint64_t, Cell> leaves;
  leaves.reserve(cells.size() * 2);
  for (size_t e = 0; e < cells.size(); ++e) {
    const Cell& c = cells[e];
    const int act = action[e];
    if (act < 0 || act > 2) throw Error(-1, "unknown refinement action");
    if (act == 1) {
      if (c.level >= 14) throw Error(-2, "refinement beyond level 14");
      for (int z = 0; z < 8; ++z) {
        Cell k{c.macro, c.level + 1, {2 * c.a[0] + (z & 1), 2 * c.a[1] + ((z >> 1) & 1), 2 * c.a[2] + (z >> 2)}, c.p};
        leaves[key_of(k.macro, k.level, k.a[0], k.a[1], k.a[2])] = k;
      }
    } else {
      Cell k = c;
      if (act == 2) k.p = std::min(c.p + 1, std::max(max_p, c.p));
      leaves[key_of(k.macro, k.level, k.a[0], k.a[1], k.a[2])] = k;
    }
  }
  balance_leaves(mm, leaves);
  for (const auto& kv : leaves)
    if (kv.second.level > 14) throw Error(-2, "refinement beyond level 14");
  // each old cell is replaced in place by the leaves inside it, children in the order of their
  // bits (x fastest)
  out.clear();
  origin.clear();
  std::vector<Cell> stack;
  for (size_t e = 0; e < cells.size(); ++e) {
    stack.assign(1, cells[e]);
    while (!stack.empty()) {
      const Cell c = stack.back();
      stack.pop_back();
      auto it = leaves.find(key_of(c.macro, c.level, c.a[0], c.a[1], c.a[2]));
      if (it != leaves.end()) {
        out.push_back(it->second);
        origin.push_back(int(e));
        continue;
      }
      if (c.level >= 14) throw Error(-2, "mesh adaptation: a cell without leaves");
      for (int z = 7; z >= 0; --z)
        stack.push_back(Cell{c.macro, c.level + 1,
                             {2 * c.a[0] + (z & 1), 2 * c.a[1] + ((z >> 1) & 1), 2 * c.a[2] + (z >> 2)}, c.p});
    }
  }
  if (out.size() != leaves.size()) throw Error(-2, "mesh adaptation: leaves outside the old cells");
}

bool cell_across(const MacroMesh& mm, const Cell& c, int f, Cell& nb, int& fb, int& orient) {
  nb = c;
  return across(mm, c.macro, c.level, c.a, f, nb.macro, nb.a, fb, orient);
}

}  // namespace hpdg
