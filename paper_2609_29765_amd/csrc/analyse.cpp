// analyse.cpp -- symbolic analysis and static plan (see analyse.hpp).
//
// Orderings follow one written rule set (the paper names RCM, AMD, METIS and
// SCOTCH without parameters, Sec. 3; the rules below are this library's):
//   * vertices of degree > max(16, floor(sqrt(100 n))) are set aside and
//     ordered last, ascending;
//   * connected components are ordered one after another, ascending by their
//     smallest vertex;
//   * pseudo-peripheral root (George-Liu): start at the minimum-degree vertex
//     (lowest index on ties), move to the minimum-degree vertex of the last
//     BFS level while that strictly increases the eccentricity;
//   * RCM: Cuthill-McKee from that root, unvisited neighbours appended by
//     (degree, index) ascending, each component's order reversed;
//   * ND: sets of at most 64 vertices, or of depth < 2, are leaves in
//     ascending order; otherwise the middle level (index ceil(depth/2)) of
//     the root's level structure is the separator, the components of the rest
//     are dissected in ascending order of their smallest vertex, then the
//     separator ascending;
//   * AUTO scores NATURAL, RCM, ND on (nnz(L), active tiles): minimum fill when
//     the natural order's mean occupancy is below 0.15, else minimum active
//     tiles unless a candidate has at most half its fill; ND wins on n >= 50000
//     when its fill is within 1.25x of the best.
// Degrees are always counted inside the set being ordered.
#include "analyse.hpp"

#include <algorithm>
#include <map>
#include <queue>
#include <thread>
#include <cmath>
#include <functional>

#include "../../include/stc.h"

namespace stc {

namespace {

struct Graph {
  std::vector<int64_t> start;
  std::vector<int32_t> nbr;
  int32_t deg(int32_t v) const { return (int32_t)(start[v + 1] - start[v]); }
};

Graph make_graph(int64_t n, const int64_t* cp, const int32_t* ri) {
  std::vector<std::vector<int32_t>> adj((size_t)n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = cp[j] + 1; p < cp[j + 1]; ++p) {
      adj[(size_t)ri[p]].push_back((int32_t)j);
      adj[(size_t)j].push_back(ri[p]);
    }
  Graph g;
  g.start.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) g.start[v + 1] = g.start[v] + (int64_t)adj[v].size();
  g.nbr.resize((size_t)g.start[n]);
  for (int64_t v = 0; v < n; ++v) {
    std::sort(adj[v].begin(), adj[v].end());
    std::copy(adj[v].begin(), adj[v].end(), g.nbr.begin() + g.start[v]);
  }
  return g;
}

int64_t dense_threshold(int64_t n) {
  // largest t with t*t <= 100 n, by bisection
  int64_t lo = 0, hi = 1;
  while (hi * hi <= 100 * n) hi *= 2;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (mid * mid <= 100 * n) lo = mid; else hi = mid;
  }
  return std::max<int64_t>(16, lo);
}

class Orderer {
 public:
  Orderer(const Graph& g, int64_t n) : g_(g), owner_((size_t)n, 0), mark_((size_t)n, 0),
                                        lvl_((size_t)n, 0) {}

  // order the vertices of `set` (ascending, owner == id) by method, appending to out
  void order_components(const std::vector<int32_t>& set, int32_t id, int method,
                        std::vector<int32_t>* out) {
    for (auto& comp : split(set, id)) {
      int32_t cid = fresh();
      for (int32_t v : comp) owner_[v] = cid;
      if (method == kRcm) rcm(comp, cid, out); else nd(comp, cid, out);
    }
  }
  int32_t fresh() { return ++ids_; }
  void set_owner(int32_t v, int32_t id) { owner_[v] = id; }

 private:
  const Graph& g_;
  std::vector<int32_t> owner_, mark_, lvl_;
  int32_t ids_ = 1, stamp_ = 0;

  int32_t degree_in(int32_t v, int32_t id) const {
    int32_t d = 0;
    for (int64_t p = g_.start[v]; p < g_.start[v + 1]; ++p) d += owner_[g_.nbr[p]] == id;
    return d;
  }

  // components of the set, each sorted, in ascending order of their minimum
  std::vector<std::vector<int32_t>> split(const std::vector<int32_t>& set, int32_t id) {
    std::vector<std::vector<int32_t>> comps;
    ++stamp_;
    for (int32_t s : set) {
      if (mark_[s] == stamp_) continue;
      std::vector<int32_t> c{s};
      mark_[s] = stamp_;
      for (size_t h = 0; h < c.size(); ++h) {
        int32_t u = c[h];
        for (int64_t p = g_.start[u]; p < g_.start[u + 1]; ++p) {
          int32_t w = g_.nbr[p];
          if (owner_[w] == id && mark_[w] != stamp_) {
            mark_[w] = stamp_;
            c.push_back(w);
          }
        }
      }
      std::sort(c.begin(), c.end());
      comps.push_back(std::move(c));
    }
    return comps;
  }

  // level structure from root; returns levels as lists
  std::vector<std::vector<int32_t>> levels_from(int32_t root, int32_t id) {
    std::vector<std::vector<int32_t>> L{{root}};
    ++stamp_;
    mark_[root] = stamp_;
    lvl_[root] = 0;
    while (true) {
      std::vector<int32_t> next;
      for (int32_t u : L.back())
        for (int64_t p = g_.start[u]; p < g_.start[u + 1]; ++p) {
          int32_t w = g_.nbr[p];
          if (owner_[w] == id && mark_[w] != stamp_) {
            mark_[w] = stamp_;
            lvl_[w] = (int32_t)L.size();
            next.push_back(w);
          }
        }
      if (next.empty()) break;
      L.push_back(std::move(next));
    }
    return L;
  }

  int32_t min_degree_vertex(const std::vector<int32_t>& vs, int32_t id) const {
    int32_t best = -1, bd = 0;
    for (int32_t v : vs) {
      int32_t d = degree_in(v, id);
      if (best < 0 || d < bd || (d == bd && v < best)) {
        best = v;
        bd = d;
      }
    }
    return best;
  }

  int32_t peripheral(const std::vector<int32_t>& comp, int32_t id,
                     std::vector<std::vector<int32_t>>* levels) {
    int32_t r = min_degree_vertex(comp, id);
    auto L = levels_from(r, id);
    for (;;) {
      int32_t v = min_degree_vertex(L.back(), id);
      auto L2 = levels_from(v, id);
      if (L2.size() > L.size()) {
        r = v;
        L = std::move(L2);
      } else {
        break;
      }
    }
    *levels = std::move(L);
    return r;
  }

  void rcm(const std::vector<int32_t>& comp, int32_t id, std::vector<int32_t>* out) {
    std::vector<std::vector<int32_t>> L;
    int32_t r = peripheral(comp, id, &L);
    std::vector<int32_t> order{r};
    ++stamp_;
    mark_[r] = stamp_;
    std::vector<std::pair<int32_t, int32_t>> cand;
    for (size_t h = 0; h < order.size(); ++h) {
      int32_t u = order[h];
      cand.clear();
      for (int64_t p = g_.start[u]; p < g_.start[u + 1]; ++p) {
        int32_t w = g_.nbr[p];
        if (owner_[w] == id && mark_[w] != stamp_) {
          mark_[w] = stamp_;
          cand.emplace_back(degree_in(w, id), w);
        }
      }
      std::sort(cand.begin(), cand.end());
      for (auto& c : cand) order.push_back(c.second);
    }
    out->insert(out->end(), order.rbegin(), order.rend());
  }

  void nd(const std::vector<int32_t>& comp, int32_t id, std::vector<int32_t>* out) {
    if (comp.size() <= 64) {
      out->insert(out->end(), comp.begin(), comp.end());
      return;
    }
    std::vector<std::vector<int32_t>> L;
    peripheral(comp, id, &L);
    int32_t depth = (int32_t)L.size() - 1;
    if (depth < 2) {
      out->insert(out->end(), comp.begin(), comp.end());
      return;
    }
    std::vector<int32_t> sep = L[(size_t)(depth + 1) / 2];
    std::sort(sep.begin(), sep.end());
    int32_t rest_id = fresh();
    std::vector<int32_t> rest;
    rest.reserve(comp.size() - sep.size());
    for (int32_t v : comp) owner_[v] = rest_id;
    for (int32_t v : sep) owner_[v] = 0;
    for (int32_t v : comp)
      if (owner_[v] == rest_id) rest.push_back(v);
    for (auto& part : split(rest, rest_id)) {
      int32_t pid = fresh();
      for (int32_t v : part) owner_[v] = pid;
      nd(part, pid, out);
    }
    out->insert(out->end(), sep.begin(), sep.end());
  }
};

std::vector<int32_t> fixed_ordering(const Graph& g, int64_t n, int method, int32_t* ndense) {
  const int64_t thr = dense_threshold(n);
  std::vector<int32_t> kept, dense, out;
  out.reserve((size_t)n);
  for (int32_t v = 0; v < (int32_t)n; ++v) (g.deg(v) > thr ? dense : kept).push_back(v);
  *ndense = (int32_t)dense.size();
  if (method == kNatural) {
    out = kept;
  } else {
    Orderer o(g, n);
    int32_t id = o.fresh();
    for (int32_t v : kept) o.set_owner(v, id);
    o.order_components(kept, id, method, &out);
  }
  out.insert(out.end(), dense.begin(), dense.end());
  return out;
}

// elimination tree (Liu, with path compression) and the row-subtree traversal
// giving the exact pattern of L, from the strictly lower rows of P A P^T
void symbolic(Symbolic* s) {
  const int64_t n = s->n;
  // rows of the permuted strictly-lower pattern: row i -> columns j < i
  std::vector<int64_t> rs((size_t)n + 1, 0);
  for (int64_t c = 0; c < n; ++c)
    for (int64_t p = s->qp[c] + 1; p < s->qp[c + 1]; ++p) {
      int32_t a = s->iperm[s->qi[p]], b = s->iperm[c];
      rs[(size_t)std::max(a, b) + 1]++;
    }
  for (int64_t i = 0; i < n; ++i) rs[i + 1] += rs[i];
  std::vector<int32_t> rc((size_t)rs[n]);
  {
    std::vector<int64_t> pos(rs.begin(), rs.end() - 1);
    for (int64_t c = 0; c < n; ++c)
      for (int64_t p = s->qp[c] + 1; p < s->qp[c + 1]; ++p) {
        int32_t a = s->iperm[s->qi[p]], b = s->iperm[c];
        rc[(size_t)pos[std::max(a, b)]++] = std::min(a, b);
      }
  }
  s->parent.assign((size_t)n, -1);
  std::vector<int32_t> anc((size_t)n, -1);
  for (int32_t i = 0; i < (int32_t)n; ++i)
    for (int64_t p = rs[i]; p < rs[i + 1]; ++p) {
      int32_t r = rc[p];
      while (r != -1 && r != i) {
        int32_t nx = anc[r];
        anc[r] = i;
        if (nx == -1) s->parent[r] = i;
        r = nx;
      }
    }
  // row i of L: every node on the tree paths from its A entries up to i
  std::vector<int32_t> mark((size_t)n, -1);
  std::vector<int64_t> ccount((size_t)n, 1);
  std::vector<int32_t> rowk;
  std::vector<int64_t> rowstart((size_t)n + 1, 0);
  for (int32_t i = 0; i < (int32_t)n; ++i) {
    mark[i] = i;
    for (int64_t p = rs[i]; p < rs[i + 1]; ++p)
      for (int32_t k = rc[p]; mark[k] != i; k = s->parent[k]) {
        mark[k] = i;
        rowk.push_back(k);
        ccount[k]++;
      }
    rowstart[i + 1] = (int64_t)rowk.size();
  }
  s->lp.assign((size_t)n + 1, 0);
  for (int64_t j = 0; j < n; ++j) s->lp[j + 1] = s->lp[j] + ccount[j];
  s->lnz = s->lp[n];
  s->li.assign((size_t)s->lnz, 0);
  std::vector<int64_t> fill(s->lp.begin(), s->lp.end() - 1);
  for (int64_t j = 0; j < n; ++j) s->li[(size_t)fill[j]++] = (int32_t)j;
  for (int32_t i = 0; i < (int32_t)n; ++i)
    for (int64_t p = rowstart[i]; p < rowstart[i + 1]; ++p) s->li[(size_t)fill[rowk[p]]++] = i;
}

int route_of(double phi, double rho, double sigma) {
  if (rho >= 0.90) return kRouteDense;
  if (phi > 2.0 && rho < 0.15) return kRouteSupernodal;
  if (rho >= 0.15 || sigma >= 20.0) return kRouteSemisparse;
  return kRouteSupernodal;
}

// The tile grid of the analysed pattern: active rows of every off-diagonal
// tile, kd, and Algorithm 1's task list.  Column j sits at grid position
// grid_pos(j) (the identity on the uniform grid).  With features set, the
// features and the route are read off this grid and fix the storage mode;
// otherwise the ones already in s are kept.
void build_grid(Symbolic* s, int nb, int mode, bool features) {
  const int64_t n = s->n;
  const int64_t npad = s->pos.empty() ? n : s->pos[(size_t)n - 1] + 1;
  const int32_t NT = (int32_t)((npad + nb - 1) / nb);
  s->nb = nb;
  s->NT = NT;
  s->npad = npad;
  s->kd.assign((size_t)NT, 0);
  auto P = [&](int64_t j) { return grid_pos(*s, j); };
  // real columns per block (the rest of a block is padding)
  std::vector<int32_t> hreal((size_t)NT, 0);
  for (int64_t j = 0; j < n; ++j) hreal[(size_t)(P(j) / nb)]++;
  // per block column: the distinct rows below the diagonal block
  std::vector<int32_t> seen((size_t)n, -1);
  std::vector<std::vector<int32_t>> colrows((size_t)NT);
  for (int64_t j = 0; j < n; ++j) {
    int32_t k = (int32_t)(P(j) / nb);
    for (int64_t p = s->lp[j]; p < s->lp[j + 1]; ++p) {
      int32_t i = s->li[p];
      if (P(i) / nb == k) {
        s->kd[k] = std::max<int32_t>(s->kd[k], (int32_t)(i - j));
      } else if (seen[i] != k) {
        seen[i] = k;
        colrows[k].push_back(i);
      }
    }
  }
  struct Raw { int32_t m, k, lo, hi, cnt; int64_t first; };
  std::vector<Raw> raw;
  std::vector<int32_t> allrows;
  int64_t sum_true = 0;
  for (int32_t k = 0; k < NT; ++k) {
    auto& v = colrows[k];
    std::sort(v.begin(), v.end());  // ascending columns are ascending positions
    size_t a = 0;
    while (a < v.size()) {
      int32_t m = (int32_t)(P(v[a]) / nb);
      size_t b = a;
      while (b < v.size() && P(v[b]) / nb == m) ++b;
      const int64_t base = (int64_t)m * nb;
      Raw r{m, k, (int32_t)(P(v[a]) - base), (int32_t)(P(v[b - 1]) - base), (int32_t)(b - a),
            (int64_t)allrows.size()};
      for (size_t x = a; x < b; ++x) allrows.push_back((int32_t)(P(v[x]) - base));
      raw.push_back(r);
      sum_true += r.cnt;
      a = b;
    }
    std::vector<int32_t>().swap(v);
  }
  const int64_t ntiles = (int64_t)raw.size();
  if (features) {
    // features and route (Sec. 5.1)
    std::vector<int32_t> rowcount((size_t)n, 0);
    for (int32_t i : s->li) rowcount[i]++;
    int64_t maxrc = *std::max_element(rowcount.begin(), rowcount.end());
    s->phi = (double)s->lnz / (double)s->qnz;
    s->rho = ntiles ? (double)sum_true / ((double)nb * (double)ntiles) : 1.0;
    s->sigma = ((double)maxrc * (double)n) / (double)s->lnz;
    s->tact = ntiles + NT;
    s->route = route_of(s->phi, s->rho, s->sigma);
    if (mode == kModeAuto) mode = s->route == kRouteDense ? kModeDense : kModeSemisparse;
    s->mode = mode;
  }
  // stored rows: full height (the block's real rows) on the dense route
  s->tiles.clear();
  s->rows.clear();
  for (const Raw& r : raw) {
    TileInfo t;
    t.m = r.m;
    t.k = r.k;
    t.true_cnt = r.cnt;
    t.roff = (int64_t)s->rows.size();
    const int32_t hm = hreal[(size_t)r.m];
    if (s->mode == kModeDense) {
      t.cnt = hm;
      t.contig = 1;
      for (int32_t x = 0; x < hm; ++x) s->rows.push_back(x);
    } else {
      t.cnt = r.cnt;
      t.contig = (int8_t)(r.hi - r.lo + 1 == r.cnt);
      s->rows.insert(s->rows.end(), allrows.begin() + r.first, allrows.begin() + r.first + r.cnt);
    }
    s->tiles.push_back(t);
  }
  // Algorithm 1 over the tile neighbourhoods N(k)
  std::vector<std::vector<int32_t>> below((size_t)NT), left((size_t)NT);
  for (const TileInfo& t : s->tiles) {
    below[t.k].push_back(t.m);
    left[t.m].push_back(t.k);
  }
  for (auto& v : left) std::sort(v.begin(), v.end());
  s->tasks.clear();
  auto push = [&](int op, int m, int k, int nn) {
    s->tasks.push_back(op);
    s->tasks.push_back(m);
    s->tasks.push_back(k);
    s->tasks.push_back(nn);
  };
  std::vector<int32_t> common;
  for (int32_t k = 0; k < NT; ++k) {
    for (int32_t nn : left[k]) push(kSyrk, -1, k, nn);
    push(kPotrf, -1, k, -1);
    for (int32_t m : below[k]) {
      common.clear();
      std::set_intersection(left[k].begin(), left[k].end(), left[m].begin(), left[m].end(),
                            std::back_inserter(common));
      for (int32_t nn : common)
        if (nn < k) push(kGemm, m, k, nn);
      push(kTrsm, m, k, -1);
    }
  }
}

int analyse_perm(Symbolic* s, int nb, int mode) {
  const int64_t n = s->n;
  s->iperm.assign((size_t)n, -1);
  for (int64_t a = 0; a < n; ++a) s->iperm[s->perm[a]] = (int32_t)a;
  symbolic(s);
  s->pos.clear();
  s->align = 0;
  build_grid(s, nb, mode, true);
  return 0;
}

}  // namespace

int check_pattern(int64_t n, const int64_t* cp, const int32_t* ri, std::string* why) {
  if (n < 1 || n >= (int64_t(1) << 31) || !cp || !ri) {
    *why = "n out of range or null pattern";
    return STC_ERR_ARG;
  }
  if (cp[0] != 0) {
    *why = "colptr[0] != 0";
    return STC_ERR_PATTERN;
  }
  for (int64_t j = 0; j < n; ++j) {
    if (cp[j + 1] <= cp[j]) {
      *why = "column " + std::to_string(j) + " has no diagonal";
      return STC_ERR_PATTERN;
    }
    if (ri[cp[j]] != j) {
      *why = "column " + std::to_string(j) + ": diagonal missing or an upper entry";
      return STC_ERR_PATTERN;
    }
    int32_t prev = (int32_t)j;
    for (int64_t p = cp[j] + 1; p < cp[j + 1]; ++p) {
      if (ri[p] <= prev || ri[p] >= n) {
        *why = "column " + std::to_string(j) + ": rows unsorted, duplicated or out of range";
        return STC_ERR_PATTERN;
      }
      prev = ri[p];
    }
  }
  return 0;
}

void build_lmap(const Symbolic& s, Plan* p) {
  const int32_t nb = s.nb, NT = s.NT;
  const int64_t ntiles = (int64_t)s.tiles.size();
  std::vector<int64_t> col_first((size_t)NT + 1, 0);
  for (const TileInfo& t : s.tiles) col_first[t.k + 1]++;
  for (int32_t k = 0; k < NT; ++k) col_first[k + 1] += col_first[k];
  std::vector<int32_t> inv((size_t)ntiles * nb, -1);
  for (int64_t t = 0; t < ntiles; ++t) {
    const TileInfo& ti = s.tiles[t];
    for (int32_t r = 0; r < ti.cnt; ++r) inv[(size_t)t * nb + s.rows[ti.roff + r]] = r;
  }
  p->lmap.resize((size_t)s.lnz);
  for (int64_t j = 0; j < s.n; ++j) {
    const int64_t pj = grid_pos(s, j);
    const int32_t bj = (int32_t)(pj / nb);
    int64_t t = col_first[bj];  // rows ascend, so the tiles of column j are met in order
    for (int64_t q = s.lp[j]; q < s.lp[j + 1]; ++q) {
      const int64_t pi = grid_pos(s, s.li[q]);
      const int32_t bi = (int32_t)(pi / nb);
      if (bi == bj) {
        p->lmap[q] = (int64_t)bj * nb * nb + (pi % nb) * nb + (pj % nb);
        continue;
      }
      while (s.tiles[t].m < bi) ++t;
      p->lmap[q] = p->tile_off[t] + (int64_t)inv[(size_t)t * nb + (pi % nb)] * nb + (pj % nb);
    }
  }
}

int analyse(int64_t n, const int64_t* cp, const int32_t* ri, int method, int nb, int mode,
            const int32_t* perm, Symbolic* out, std::string* why) {
  int rc = check_pattern(n, cp, ri, why);
  if (rc) return rc;
  if (nb < 1 || method < kNatural || method > kGiven || mode < kModeAuto || mode > kModeSemisparse) {
    *why = "invalid nb, ordering or mode";
    return STC_ERR_ARG;
  }
  auto fresh = [&]() {
    Symbolic s;
    s.n = n;
    s.qnz = cp[n];
    s.qp.assign(cp, cp + n + 1);
    s.qi.assign(ri, ri + cp[n]);
    return s;
  };
  if (method == kGiven) {
    if (!perm) {
      *why = "ordering GIVEN without a permutation";
      return STC_ERR_ARG;
    }
    std::vector<char> hit((size_t)n, 0);
    for (int64_t a = 0; a < n; ++a) {
      if (perm[a] < 0 || perm[a] >= n || hit[perm[a]]) {
        *why = "given permutation is not a permutation of 0..n-1";
        return STC_ERR_ARG;
      }
      hit[perm[a]] = 1;
    }
    *out = fresh();
    out->perm.assign(perm, perm + n);
    out->method = kGiven;
    return analyse_perm(out, nb, mode);
  }
  Graph g = make_graph(n, cp, ri);
  if (method != kAuto) {
    *out = fresh();
    out->perm = fixed_ordering(g, n, method, &out->ndense);
    out->method = method;
    return analyse_perm(out, nb, mode);
  }
  // the three candidates are independent: each is ordered and scored on a
  // thread of its own, as the paper runs its candidate orderings in
  // parallel (Sec. 3); the choice below reads only their scores
  Symbolic cand[3];
  int crc[3] = {0, 0, 0};
  auto score = [&](int m) {
    try {
      cand[m] = fresh();
      cand[m].perm = fixed_ordering(g, n, m, &cand[m].ndense);
      cand[m].method = m;
      crc[m] = analyse_perm(&cand[m], nb, mode);
    } catch (const std::bad_alloc&) {
      crc[m] = STC_ERR_ALLOC;
    }
  };
  {
    std::thread t1(score, 1), t2(score, 2);
    score(0);
    t1.join();
    t2.join();
  }
  for (int m = 0; m < 3; ++m)
    if (crc[m]) {
      *why = "analysis of an ordering candidate failed";
      return crc[m];
    }
  int best_fill = 0;
  for (int m = 1; m < 3; ++m)
    if (cand[m].lnz < cand[best_fill].lnz) best_fill = m;
  int win;
  if (cand[kNatural].rho < 0.15) {
    win = best_fill;
  } else {
    int best_t = 0;
    for (int m = 1; m < 3; ++m)
      if (cand[m].tact < cand[best_t].tact) best_t = m;
    win = best_t;
    int low = -1;
    for (int m = 0; m < 3; ++m)
      if (2 * cand[m].lnz <= cand[best_t].lnz && (low < 0 || cand[m].lnz < cand[low].lnz)) low = m;
    if (low >= 0) win = low;
  }
  if (n >= 50000 && 4 * cand[kNd].lnz <= 5 * cand[best_fill].lnz) win = kNd;
  *out = std::move(cand[win]);
  return 0;
}

void align_tiles(Symbolic* s, int64_t min_subtree) {
  const int64_t n = s->n;
  const int32_t nb = s->nb;
  s->pos.clear();
  s->align = 0;
  if (min_subtree > 0) {
    // subtree sizes and first columns (a child precedes its parent)
    std::vector<int64_t> size((size_t)n, 1), first((size_t)n);
    for (int64_t j = 0; j < n; ++j) first[(size_t)j] = j;
    for (int64_t j = 0; j < n; ++j) {
      const int32_t q = s->parent[(size_t)j];
      if (q < 0) continue;
      size[(size_t)q] += size[(size_t)j];
      first[(size_t)q] = std::min(first[(size_t)q], first[(size_t)j]);
    }
    // a large subtree whose columns are consecutive starts a tile
    std::vector<char> start((size_t)n, 0);
    for (int64_t r = 0; r < n; ++r)
      if (size[(size_t)r] >= min_subtree && first[(size_t)r] == r - size[(size_t)r] + 1) start[(size_t)first[(size_t)r]] = 1;
    s->pos.resize((size_t)n);
    int64_t cur = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (start[(size_t)j] && cur % nb) cur += nb - cur % nb;
      s->pos[(size_t)j] = cur++;
    }
    s->align = min_subtree;
  }
  build_grid(s, nb, s->mode, false);
}

// ---------------------------------------------------------------------------
// execution plan
// ---------------------------------------------------------------------------

namespace {

// Memory of the split-K partial slots.  A slot is live from the kernel that
// writes it (its split task's, level L, early groups) to the kernel that
// folds it (its partner's, a later level).  Slots share memory: a slot may
// take memory that earlier slots used once the kernel that folded each of
// them is an ancestor, in the kernel graph, of the kernel that writes the new
// slot.  The graph then orders every access to the shared memory with the
// edges it has anyway, so sharing adds no edge and costs no overlap.  The
// slots are placed first-fit in the order of their writing kernels; the
// memory is kept as segments that cover [0, parts), each owned by the last
// slot placed on it (a slot placed after that one's fold is also placed after
// the folds of all earlier owners, which precede that slot's writer).
void place_slots(Plan* p) {
  std::vector<KernelNode> dag;
  kernel_dag(*p, &dag);
  const size_t N = dag.size(), W = N / 64 + 1;
  std::vector<uint64_t> anc(N * W, 0);
  for (size_t x = 0; x < N; ++x)
    for (int32_t d : dag[x].deps) {
      for (size_t w = 0; w < W; ++w) anc[x * W + w] |= anc[(size_t)d * W + w];
      anc[x * W + (size_t)d / 64] |= uint64_t(1) << (d % 64);
    }
  std::map<std::pair<int32_t, int32_t>, int32_t> node_of;
  for (size_t x = 0; x < N; ++x) node_of[{dag[x].level, dag[x].kind}] = (int32_t)x;
  // kernel of each update task: the last groups lead each list of items and
  // form kind 3 where the level launches them apart, the rest kind 1
  std::vector<int32_t> node_of_task(p->upd.size(), -1);
  for (int32_t L = 0; L < (int32_t)p->levels.size(); ++L) {
    const Level& lv = p->levels[(size_t)L];
    for (const std::vector<int32_t>* v : {&lv.big_items, &lv.upd_items}) {
      const size_t nl = 4 * (size_t)(v == &lv.big_items ? lv.big_last : lv.upd_last);
      for (size_t q = 0; q < v->size(); q += 4) node_of_task[(size_t)(*v)[q]] = node_of.at({L, q < nl ? 3 : 1});
    }
  }
  std::vector<int32_t> split;
  for (int32_t id = 0; id < (int32_t)p->upd.size(); ++id)
    if (p->upd[(size_t)id].nsplit > 1) split.push_back(id);
  std::stable_sort(split.begin(), split.end(), [&](int32_t a, int32_t b) {
    return node_of_task[(size_t)a] < node_of_task[(size_t)b];
  });
  struct Seg {
    int64_t lo, hi;
    int32_t task;
  };
  std::vector<Seg> segs, next;
  int64_t end = 0;
  for (int32_t id : split) {
    UpdTask& u = p->upd[(size_t)id];
    const int64_t need = (int64_t)(u.nsplit - 1) * u.c_rows * p->nb;
    const int32_t wnode = node_of_task[(size_t)id];
    auto freed = [&](const Seg& g) {
      const int32_t f = node_of_task[(size_t)p->upd[(size_t)g.task].partner];
      return (anc[(size_t)wnode * W + (size_t)f / 64] >> (f % 64)) & 1;
    };
    // lowest start of a run of freed segments that holds the slot; a run
    // that reaches the end continues into new memory
    int64_t start = end;
    for (size_t i = 0; i < segs.size();) {
      if (!freed(segs[i])) {
        ++i;
        continue;
      }
      size_t j = i;
      while (j < segs.size() && freed(segs[j]) && segs[j].hi - segs[i].lo < need) ++j;
      if (j == segs.size() || freed(segs[j])) {
        start = segs[i].lo;
        break;
      }
      i = j + 1;
    }
    const int64_t stop = start + need;
    next.clear();
    bool placed = false;
    for (const Seg& g : segs) {
      if (g.hi <= start || g.lo >= stop) {
        if (g.lo >= stop && !placed) {
          next.push_back({start, stop, id});
          placed = true;
        }
        next.push_back(g);
        continue;
      }
      if (g.lo < start) next.push_back({g.lo, start, g.task});
      if (!placed) {
        next.push_back({start, stop, id});
        placed = true;
      }
      if (g.hi > stop) next.push_back({stop, g.hi, g.task});
    }
    if (!placed) next.push_back({start, stop, id});
    segs.swap(next);
    end = std::max(end, stop);
    u.part_off = start;
    p->upd[(size_t)u.partner].in_part_off = start;
  }
  p->parts = end;
}

}  // namespace

// 448 for tiles of 128 and 256 (two 128-block work-groups fit a compute
// unit), 896 for smaller tiles, whose 64-block work-groups fit several to a
// compute unit (both the best of sweeps on MI355X)
int64_t default_wg_slots(int nb) { return nb <= 64 ? 896 : 448; }

int build_plan(const Symbolic& s, int bm, int br, int64_t wg_slots, Plan* p, std::string* why, int max_split,
               int fold_pct) {
  const int32_t nb = s.nb, NT = s.NT;
  const int64_t n = s.n;
  (void)why;
  *p = Plan();
  p->wg_slots = wg_slots > 0 ? wg_slots : default_wg_slots(nb);
  if (max_split > 0) p->max_split = max_split;
  if (fold_pct > 0) p->fold_pct = fold_pct;
  p->nb = nb;
  p->NT = NT;
  p->bm = bm;
  p->br = br;
  const int64_t ntiles = (int64_t)s.tiles.size();
  // tile store: diagonal tiles first (nb x nb, row-major), then the packed
  // off-diagonal tiles (stored rows x nb, row-major)
  int64_t off = (int64_t)NT * nb * nb;
  p->tile_off.resize((size_t)ntiles);
  for (int64_t t = 0; t < ntiles; ++t) {
    p->tile_off[t] = off;
    off += (int64_t)s.tiles[t].cnt * nb;
  }
  p->store = off;
  // real columns of each diagonal tile: a prefix of its positions, the
  // rest padding (identity in the store)
  p->diag_h.assign((size_t)NT, 0);
  for (int64_t j = 0; j < n; ++j) p->diag_h[(size_t)(grid_pos(s, j) / nb)]++;
  // tile lookup per block column: (m -> tile index), and inverse row maps
  std::vector<int64_t> col_first((size_t)NT + 1, 0);
  for (const TileInfo& t : s.tiles) col_first[t.k + 1]++;
  for (int32_t k = 0; k < NT; ++k) col_first[k + 1] += col_first[k];
  auto find_tile = [&](int32_t m, int32_t k) -> int64_t {
    int64_t lo = col_first[k], hi = col_first[k + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (s.tiles[mid].m < m) lo = mid + 1; else hi = mid;
    }
    return (lo < col_first[k + 1] && s.tiles[lo].m == m) ? lo : -1;
  };
  std::vector<int32_t> inv((size_t)ntiles * nb, -1);
  for (int64_t t = 0; t < ntiles; ++t) {
    const TileInfo& ti = s.tiles[t];
    for (int32_t r = 0; r < ti.cnt; ++r) inv[(size_t)t * nb + s.rows[ti.roff + r]] = r;
  }
  auto store_pos = [&](int32_t i, int32_t j) -> int64_t {  // permuted, i >= j
    const int64_t pi = grid_pos(s, i), pj = grid_pos(s, j);
    const int32_t bi = (int32_t)(pi / nb), bj = (int32_t)(pj / nb);
    if (bi == bj) return (int64_t)bj * nb * nb + (pi % nb) * nb + (pj % nb);
    int64_t t = find_tile(bi, bj);
    int32_t r = inv[(size_t)t * nb + (pi % nb)];
    return p->tile_off[t] + (int64_t)r * nb + (pj % nb);
  };
  p->vmap.resize((size_t)s.qnz);
  for (int64_t c = 0; c < n; ++c)
    for (int64_t q = s.qp[c]; q < s.qp[c + 1]; ++q) {
      int32_t a = s.iperm[s.qi[q]], b = s.iperm[c];
      p->vmap[q] = store_pos(std::max(a, b), std::min(a, b));
    }
  build_lmap(s, p);

  // gather maps: inverse row map of every tile (used as column maps), stored
  // once; identity for full tiles
  std::vector<int32_t> colmap_of((size_t)ntiles, -1);
  auto full = [&](int64_t t) {
    const TileInfo& ti = s.tiles[t];
    const int32_t hm = p->diag_h[(size_t)ti.m];
    return ti.cnt == hm && hm == nb;
  };
  for (int64_t t = 0; t < ntiles; ++t) {
    if (full(t)) continue;
    colmap_of[t] = (int32_t)p->maps.size();
    p->maps.insert(p->maps.end(), inv.begin() + t * nb, inv.begin() + (t + 1) * nb);
  }
  p->tile_imap = colmap_of;

  // fused update tasks from Algorithm 1's list, and the level schedule
  std::vector<int32_t> lvT((size_t)ntiles, -1), lvP((size_t)NT, -1);
  std::vector<int32_t> lvU_diag((size_t)NT, -1), lvU_tile((size_t)ntiles, -1);
  std::vector<int32_t> trsm_of_tile((size_t)ntiles, -1);
  double flops = 0;
  const auto& T = s.tasks;
  const size_t ntask = T.size() / 4;
  auto level_at = [&](int32_t L) -> Level& {
    if ((int32_t)p->levels.size() <= L) p->levels.resize((size_t)L + 1);
    return p->levels[(size_t)L];
  };
  // Each output tile's contributions split into an early group (operands
  // ready before the latest one) and a last group.  Both are placed as late
  // as their consumer allows: the last group one level before the TRSM (or
  // POTRF) that reads the tile, the early group one level before that.  On a
  // dense grid this puts POTRF(k) beside the n = k-1 updates of column k and
  // the bulk of column k's updates one level earlier.
  auto emit_group = [&](const std::vector<Contrib>& cs, int64_t c_off, int32_t c_rows, bool diag,
                        int32_t level) -> int32_t {
    if (cs.empty()) return -1;
    UpdTask u;
    u.c_off = c_off;
    u.c_rows = c_rows;
    u.diag = diag ? 1 : 0;
    u.c_begin = (int32_t)p->contribs.size();
    p->contribs.insert(p->contribs.end(), cs.begin(), cs.end());
    u.c_end = (int32_t)p->contribs.size();
    u.level = level;
    u.big = (nb >= 128 && c_rows >= 96) ? 1 : 0;
    p->bytes_update += 16.0 * c_rows * (diag ? c_rows : nb);
    Level& lv = level_at(level);
    for (const Contrib& c : cs) {
      const double f = diag ? (double)c.b_rows * c.b_rows * nb : 2.0 * c.a_rows * c.b_rows * nb;
      lv.flops += f;
      lv.flops_upd += f;
    }
    p->upd.push_back(u);
    return (int32_t)p->upd.size() - 1;
  };
  std::vector<Contrib> run;
  std::vector<int32_t> ready;
  size_t a = 0;
  while (a < ntask) {
    int op = T[4 * a], m = T[4 * a + 1], k = T[4 * a + 2];
    if (op == kSyrk || op == kGemm) {
      const bool diag = op == kSyrk;
      int64_t tout = diag ? -1 : find_tile(m, k);
      run.clear();
      ready.clear();
      size_t b = a;
      for (; b < ntask && T[4 * b] == op && T[4 * b + 1] == m && T[4 * b + 2] == k; ++b) {
        int nn = T[4 * b + 3];
        Contrib c;
        int64_t tb = find_tile(k, nn);
        c.b_off = p->tile_off[tb];
        c.b_rows = s.tiles[tb].cnt;
        c.colmap = colmap_of[tb];
        if (diag) {
          c.a_off = c.b_off;
          c.a_rows = c.b_rows;
          c.rowmap = colmap_of[tb];
          ready.push_back(lvT[tb] + 1);
          flops += (double)s.tiles[tb].cnt * s.tiles[tb].cnt * nb;
          p->flops_update += (double)s.tiles[tb].cnt * s.tiles[tb].cnt * nb;
          p->bytes_update += 8.0 * s.tiles[tb].cnt * nb;
        } else {
          int64_t ta = find_tile(m, nn);
          c.a_off = p->tile_off[ta];
          c.a_rows = s.tiles[ta].cnt;
          const TileInfo& to = s.tiles[tout];
          const TileInfo& tia = s.tiles[ta];
          bool same = to.cnt == tia.cnt &&
                      std::equal(s.rows.begin() + to.roff, s.rows.begin() + to.roff + to.cnt,
                                 s.rows.begin() + tia.roff);
          if (same) {
            c.rowmap = -1;
          } else {
            c.rowmap = (int32_t)p->maps.size();
            for (int32_t r = 0; r < to.cnt; ++r)
              p->maps.push_back(inv[(size_t)ta * nb + s.rows[to.roff + r]]);
          }
          ready.push_back(std::max(lvT[ta], lvT[tb]) + 1);
          flops += 2.0 * tia.cnt * s.tiles[tb].cnt * nb;
          p->flops_update += 2.0 * tia.cnt * s.tiles[tb].cnt * nb;
          p->bytes_update += 8.0 * (tia.cnt + s.tiles[tb].cnt) * nb;
        }
        run.push_back(c);
      }
      const int32_t rl = *std::max_element(ready.begin(), ready.end());
      std::vector<Contrib> early, last;
      int32_t re = 0;  // readiness of the early group
      for (size_t x = 0; x < run.size(); ++x) {
        if (ready[x] == rl) {
          last.push_back(run[x]);
        } else {
          early.push_back(run[x]);
          re = std::max(re, ready[x]);
        }
      }
      // the early group goes to the latest level of its window [re, hi] that
      // holds a POTRF, so that the single-work-group factorization runs beside
      // it; otherwise to hi
      auto early_level = [&](int32_t hi) {
        for (int32_t L = hi; L >= re; --L)
          if (L < (int32_t)p->levels.size() && !p->levels[(size_t)L].potrf.empty()) return L;
        return hi;
      };
      if (diag) {
        lvU_diag[k] = rl;  // POTRF(k) follows at rl + 1
        int32_t e = emit_group(early, (int64_t)k * nb * nb, p->diag_h[k], true, early_level(rl - 1));
        int32_t l = emit_group(last, (int64_t)k * nb * nb, p->diag_h[k], true, rl);
        if (e >= 0) p->upd[(size_t)e].partner = l;
      } else {
        // the TRSM of this tile waits for both the updates and POTRF(k)
        const int32_t lt = std::max(rl, lvP[k]) + 1;
        lvU_tile[tout] = lt - 1;
        const int64_t off = p->tile_off[tout];
        const int32_t rows = s.tiles[tout].cnt;
        int32_t e = emit_group(early, off, rows, false, early_level(lt - 2));
        int32_t l = emit_group(last, off, rows, false, lt - 1);
        if (e >= 0) p->upd[(size_t)e].partner = l;
      }
      a = b;
    } else if (op == kPotrf) {
      lvP[k] = lvU_diag[k] + 1;  // 0 when nothing updates the diagonal tile
      level_at(lvP[k]).potrf.push_back(k);
      level_at(lvP[k]).flops += (double)p->diag_h[k] * p->diag_h[k] * p->diag_h[k] / 3.0;
      level_at(lvP[k]).flops_potrf += (double)p->diag_h[k] * p->diag_h[k] * p->diag_h[k] / 3.0;
      flops += (double)p->diag_h[k] * p->diag_h[k] * p->diag_h[k] / 3.0;
      p->flops_potrf += (double)p->diag_h[k] * p->diag_h[k] * p->diag_h[k] / 3.0;
      ++a;
    } else {  // kTrsm
      int64_t t = find_tile(m, k);
      TrsmTask tt;
      tt.x_off = p->tile_off[t];
      tt.l_off = (int64_t)k * nb * nb;
      tt.rows = s.tiles[t].cnt;
      tt.k = k;
      int32_t id = (int32_t)p->trsm.size();
      p->trsm.push_back(tt);
      trsm_of_tile[t] = id;
      lvT[t] = std::max(lvU_tile[t], lvP[k]) + 1;
      Level& L = level_at(lvT[t]);
      L.flops += (double)tt.rows * nb * nb;
      L.flops_trsm += (double)tt.rows * nb * nb;
      for (int32_t x = 0; x < (tt.rows + br - 1) / br; ++x) {
        L.trsm_items.push_back(id);
        L.trsm_items.push_back(x);
      }
      flops += (double)tt.rows * nb * nb;
      p->flops_trsm += (double)tt.rows * nb * nb;
      ++a;
    }
  }
  // work items; early groups of large tiles in under-filled levels split
  // their contribution range (deterministic: partial slots folded in by the
  // tile's last group)
  {
    const int32_t nlev = (int32_t)p->levels.size();
    std::vector<int64_t> items((size_t)nlev, 0);
    auto blocks = [&](const UpdTask& u) -> int64_t {
      const int32_t b = u.big ? 128 : bm;
      const int64_t nr = (u.c_rows + b - 1) / b;
      return u.diag ? nr * (nr + 1) / 2 : nr * ((nb + b - 1) / b);
    };
    // a level with few 128-blocks runs them as 64-blocks: four times the
    // work-groups for the same work
    std::vector<int64_t> bigblocks((size_t)nlev, 0);
    for (const UpdTask& u : p->upd)
      if (u.big) bigblocks[(size_t)u.level] += blocks(u);
    for (UpdTask& u : p->upd)
      if (u.big && bigblocks[(size_t)u.level] < 64 && u.c_end - u.c_begin <= 2) u.big = 0;
    // Split of the early groups' K streams.  The update kernels run a task
    // as one stream of (contribution, 16-wide K chunk) steps, nb / 16 per
    // contribution, so a task can be cut at any step; a part is at least
    // kMinPart steps, and parts s > 0 leave partial slots that the task's
    // partner (its tile's next update, at a later level) folds in.  A
    // level's split is chosen among two families -- every splittable task
    // in s parts (s = 1..16, then every 4th up to 32 and every 8th up to
    // max_split), or every splittable task cut into parts of at
    // most 8 t steps (t = 1..16) -- by the estimated makespan of the level
    // plus those of the levels holding the partners it affects.  Makespans
    // come from simulating longest-first list scheduling of a level's items
    // on wg_slots concurrent work-groups.  Two passes over the levels in
    // order; the second sees the first pass's splits of later levels.
    // Item durations are in units of one 128-block contribution; a 64-block
    // contribution is a quarter; the epilogue costs a quarter, and each
    // folded partial slot 0.45 (128-block) or 0.12 (64-block) -- measured
    // on MI355X, where folding a 128-block slot takes about half the time of
    // one contribution -- times fold_pct percent (a schedule option: how
    // much a fold costs depends on how loaded the device is around it).
    (void)items;
    const int64_t ksteps = std::max<int64_t>(1, nb / 16);
    constexpr int64_t kMinPart = 8;
    auto steps_of = [&](const UpdTask& u) { return (int64_t)(u.c_end - u.c_begin) * ksteps; };
    auto max_parts = [&](const UpdTask& u) -> int32_t {
      return u.partner >= 0 ? (int32_t)std::max<int64_t>(1, std::min<int64_t>(p->max_split, steps_of(u) / kMinPart)) : 1;
    };
    auto dur = [&](const UpdTask& u, int64_t steps_part) {
      return (u.big ? 1.0 : 0.25) * (double)steps_part / (double)ksteps + 0.25 +
             (u.big ? 0.45 : 0.12) * 0.01 * p->fold_pct * u.in_npart;
    };
    std::vector<std::vector<int32_t>> lev_tasks((size_t)nlev);
    for (int32_t id = 0; id < (int32_t)p->upd.size(); ++id) lev_tasks[(size_t)p->upd[(size_t)id].level].push_back(id);
    const int64_t slots = p->wg_slots;
    std::vector<double> durs;
    // estimated makespan of level L with the tasks' current nsplit / in_npart
    auto makespan = [&](int32_t L) {
      durs.clear();
      for (int32_t id : lev_tasks[(size_t)L]) {
        const UpdTask& u = p->upd[(size_t)id];
        const int64_t tot = steps_of(u), nblk = blocks(u);
        for (int32_t part = 0; part < u.nsplit; ++part) {
          const double d = dur(u, tot * (part + 1) / u.nsplit - tot * part / u.nsplit);
          for (int64_t b = 0; b < nblk; ++b) durs.push_back(d);
        }
      }
      if (durs.empty()) return 0.0;
      std::sort(durs.begin(), durs.end(), std::greater<double>());
      std::priority_queue<double, std::vector<double>, std::greater<double>> q;
      for (int64_t x = 0; x < std::min<int64_t>(slots, (int64_t)durs.size()); ++x) q.push(0.0);
      double mk = 0;
      for (double d : durs) {
        const double t = q.top() + d;
        q.pop();
        q.push(t);
        mk = std::max(mk, t);
      }
      return mk;
    };
    auto apply = [&](const std::vector<int32_t>& ids, const std::vector<int32_t>& sp) {
      for (size_t x = 0; x < ids.size(); ++x) {
        UpdTask& u = p->upd[(size_t)ids[x]];
        u.nsplit = sp[x];
        if (u.partner >= 0) p->upd[(size_t)u.partner].in_npart = sp[x] - 1;
      }
    };
    std::vector<int32_t> cand, best_s, plev;
    for (int32_t pass = 0; pass < 2; ++pass)
      for (int32_t L = 0; L < nlev; ++L) {
        const std::vector<int32_t>& ids = lev_tasks[(size_t)L];
        bool any = false;
        plev.clear();
        for (int32_t id : ids) {
          const UpdTask& u = p->upd[(size_t)id];
          if (max_parts(u) > 1) {
            any = true;
            plev.push_back(p->upd[(size_t)u.partner].level);
          }
        }
        if (!any) continue;
        std::sort(plev.begin(), plev.end());
        plev.erase(std::unique(plev.begin(), plev.end()), plev.end());
        double best = 1e300;
        for (int32_t fam = 0; fam < 2; ++fam)
          for (int32_t c = 1; c <= (fam == 0 ? std::max<int32_t>(16, p->max_split) : 16); c += (c < 16 ? 1 : c < 32 ? 4 : 8)) {
            cand.assign(ids.size(), 1);
            for (size_t x = 0; x < ids.size(); ++x) {
              const UpdTask& u = p->upd[(size_t)ids[x]];
              const int64_t want = fam == 0 ? c : (steps_of(u) + c * kMinPart - 1) / (c * kMinPart);
              cand[x] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(want, max_parts(u)));
            }
            apply(ids, cand);
            double cost = makespan(L);
            for (int32_t l2 : plev) cost += makespan(l2);
            if (cost < best - 1e-9) {
              best = cost;
              best_s = cand;
            }
          }
        apply(ids, best_s);
      }
    for (UpdTask& u : p->upd) {
      if (u.nsplit < 2) continue;
      UpdTask& l = p->upd[(size_t)u.partner];
      l.in_npart = u.nsplit - 1;
    }
    for (int32_t id = 0; id < (int32_t)p->upd.size(); ++id) {
      const UpdTask& u = p->upd[(size_t)id];
      const int32_t b = u.big ? 128 : bm;
      const int32_t nbr = (u.c_rows + b - 1) / b, nbc = u.diag ? nbr : (nb + b - 1) / b;
      auto& dst = u.big ? p->levels[(size_t)u.level].big_items : p->levels[(size_t)u.level].upd_items;
      for (int32_t part = 0; part < u.nsplit; ++part)
        for (int32_t x = 0; x < nbr; ++x)
          for (int32_t y = 0; y < nbc; ++y) {
            if (u.diag && y > x) continue;
            dst.push_back(id);
            dst.push_back(x);
            dst.push_back(y);
            dst.push_back(part);
          }
    }
    // longest items first: work-groups are dispatched in index order, so a
    // level runs as a longest-processing-time-first list schedule
    auto item_dur = [&](const int32_t* q) {
      const UpdTask& u = p->upd[(size_t)q[0]];
      const int64_t tot = steps_of(u);
      return dur(u, tot * (q[3] + 1) / u.nsplit - tot * q[3] / u.nsplit);
    };
    for (Level& L : p->levels) {
      double w_big_early = 0, w_upd_early = 0;
      for (std::vector<int32_t>* v : {&L.big_items, &L.upd_items}) {
        const size_t cnt = v->size() / 4;
        std::vector<size_t> order(cnt);
        for (size_t x = 0; x < cnt; ++x) order[x] = x;
        // last groups first (their consumers are in the next level), each
        // part longest first
        auto early = [&](size_t x) { return p->upd[(size_t)(*v)[4 * x]].partner >= 0; };
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
          if (early(a) != early(b)) return early(b);
          return item_dur(&(*v)[4 * a]) > item_dur(&(*v)[4 * b]);
        });
        int32_t nlast = 0;
        double w_early = 0;
        for (size_t x = 0; x < cnt; ++x) {
          nlast += early(x) ? 0 : 1;
          if (early(x)) w_early += item_dur(&(*v)[4 * x]);
        }
        (v == &L.big_items ? L.big_last : L.upd_last) = nlast;
        (v == &L.big_items ? w_big_early : w_upd_early) = w_early;
        std::vector<int32_t> out(v->size());
        for (size_t x = 0; x < cnt; ++x)
          std::copy(v->begin() + 4 * order[x], v->begin() + 4 * order[x] + 4, out.begin() + 4 * x);
        v->swap(out);
      }
      // the last groups get a launch of their own (so that the next level's
      // TRSM / POTRF need not wait for the early groups) only when the early
      // groups fill at least one round of the device; otherwise one launch
      if (w_big_early + w_upd_early < (double)p->wg_slots) L.big_last = L.upd_last = 0;
    }
  }
  place_slots(p);
  p->flops_tile = flops;
  for (int64_t j = 0; j < n; ++j) {
    double c = (double)(s.lp[j + 1] - s.lp[j]);
    p->flops_exact += c * c;
  }

  // solve schedule: block rows / columns and their dependency levels
  p->row_tiles_ptr.assign((size_t)NT + 1, 0);
  p->col_tiles_ptr.assign((size_t)NT + 1, 0);
  for (const TileInfo& t : s.tiles) {
    p->row_tiles_ptr[t.m + 1]++;
    p->col_tiles_ptr[t.k + 1]++;
  }
  for (int32_t k = 0; k < NT; ++k) {
    p->row_tiles_ptr[k + 1] += p->row_tiles_ptr[k];
    p->col_tiles_ptr[k + 1] += p->col_tiles_ptr[k];
  }
  p->row_tiles.resize((size_t)ntiles);
  p->col_tiles.resize((size_t)ntiles);
  {
    std::vector<int32_t> fr(p->row_tiles_ptr.begin(), p->row_tiles_ptr.end() - 1);
    std::vector<int32_t> fc(p->col_tiles_ptr.begin(), p->col_tiles_ptr.end() - 1);
    for (int64_t t = 0; t < ntiles; ++t) {
      p->row_tiles[fr[s.tiles[t].m]++] = (int32_t)t;
      p->col_tiles[fc[s.tiles[t].k]++] = (int32_t)t;
    }
  }
  std::vector<int32_t> fl((size_t)NT, 0), bl((size_t)NT, 0);
  int32_t fmax = 0, bmax = 0;
  for (int32_t m = 0; m < NT; ++m) {
    for (int32_t x = p->row_tiles_ptr[m]; x < p->row_tiles_ptr[m + 1]; ++x)
      fl[m] = std::max(fl[m], fl[s.tiles[p->row_tiles[x]].k] + 1);
    fmax = std::max(fmax, fl[m]);
  }
  for (int32_t k = NT - 1; k >= 0; --k) {
    for (int32_t x = p->col_tiles_ptr[k]; x < p->col_tiles_ptr[k + 1]; ++x)
      bl[k] = std::max(bl[k], bl[s.tiles[p->col_tiles[x]].m] + 1);
    bmax = std::max(bmax, bl[k]);
  }
  auto bucket = [&](const std::vector<int32_t>& lv, int32_t mx, std::vector<int32_t>* ptr,
                    std::vector<int32_t>* blk) {
    ptr->assign((size_t)mx + 2, 0);
    for (int32_t k = 0; k < NT; ++k) (*ptr)[lv[k] + 1]++;
    for (int32_t L = 0; L <= mx; ++L) (*ptr)[L + 1] += (*ptr)[L];
    blk->resize((size_t)NT);
    std::vector<int32_t> f(ptr->begin(), ptr->end() - 1);
    for (int32_t k = 0; k < NT; ++k) (*blk)[f[lv[k]]++] = k;
  };
  bucket(fl, fmax, &p->fwd_level_ptr, &p->fwd_level_blk);
  bucket(bl, bmax, &p->bwd_level_ptr, &p->bwd_level_blk);
  return 0;
}


// ---------------------------------------------------------------------------
// backward plan
// ---------------------------------------------------------------------------

void kernel_dag(const Plan& p, std::vector<KernelNode>* out) {
  out->clear();
  // data objects: tiles by store offset, and partial slots by split task
  // (keys -1 - task)
  std::map<int64_t, int32_t> last_writer;
  std::map<int64_t, std::vector<int32_t>> readers;
  std::vector<std::vector<uint64_t>> reach;  // ancestors of each node, bitset
  std::vector<int64_t> rd, wr;
  std::vector<std::pair<std::vector<int64_t>, std::vector<int64_t>>> acc;  // per node of the level
  std::vector<int32_t> split_src(p.upd.size(), -1);  // task -> split task whose slots it folds
  for (int32_t e = 0; e < (int32_t)p.upd.size(); ++e)
    if (p.upd[(size_t)e].nsplit > 1 && p.upd[(size_t)e].partner >= 0) split_src[(size_t)p.upd[(size_t)e].partner] = e;
  for (int32_t L = 0; L < (int32_t)p.levels.size(); ++L) {
    const Level& lv = p.levels[(size_t)L];
    const int32_t first = (int32_t)out->size();
    acc.clear();
    for (int32_t kind = 0; kind < 4; ++kind) {
      rd.clear();
      wr.clear();
      // item ranges of the update kinds: last groups lead each list
      auto lo = [&](const std::vector<int32_t>* v) {
        return kind == 3 ? (size_t)0 : 4 * (size_t)(v == &lv.big_items ? lv.big_last : lv.upd_last);
      };
      auto hi = [&](const std::vector<int32_t>* v) {
        return kind == 1 ? v->size() : 4 * (size_t)(v == &lv.big_items ? lv.big_last : lv.upd_last);
      };
      if (kind == 0) {
        for (int32_t k : lv.potrf) wr.push_back((int64_t)k * p.nb * p.nb);
      } else if (kind == 1 || kind == 3) {
        for (const std::vector<int32_t>* v : {&lv.big_items, &lv.upd_items})
          for (size_t x = lo(v); x < hi(v); x += 4) {
            const int32_t id = (*v)[x];
            const UpdTask& u = p.upd[(size_t)id];
            wr.push_back(u.c_off);
            for (int32_t c = u.c_begin; c < u.c_end; ++c) {
              rd.push_back(p.contribs[(size_t)c].a_off);
              rd.push_back(p.contribs[(size_t)c].b_off);
            }
            if (u.nsplit > 1) wr.push_back(-1 - (int64_t)id);
          }
        // partial slots folded in by a partner: the split task that names it
        for (const std::vector<int32_t>* v : {&lv.big_items, &lv.upd_items})
          for (size_t x = lo(v); x < hi(v); x += 4) {
            const int32_t e = split_src[(size_t)(*v)[x]];
            if (e >= 0) rd.push_back(-1 - (int64_t)e);
          }
      } else {
        for (size_t x = 0; x < lv.trsm_items.size(); x += 2) {
          const TrsmTask& t = p.trsm[(size_t)lv.trsm_items[x]];
          rd.push_back(t.l_off);
          wr.push_back(t.x_off);
        }
      }
      if (rd.empty() && wr.empty()) continue;
      std::sort(rd.begin(), rd.end());
      rd.erase(std::unique(rd.begin(), rd.end()), rd.end());
      std::sort(wr.begin(), wr.end());
      wr.erase(std::unique(wr.begin(), wr.end()), wr.end());
      KernelNode nd;
      nd.level = L;
      nd.kind = kind;
      std::vector<int32_t> cand;
      for (int64_t o : rd) {
        auto it = last_writer.find(o);
        if (it != last_writer.end()) cand.push_back(it->second);
      }
      for (int64_t o : wr) {
        auto it = last_writer.find(o);
        if (it != last_writer.end()) cand.push_back(it->second);
        auto jt = readers.find(o);
        if (jt != readers.end()) cand.insert(cand.end(), jt->second.begin(), jt->second.end());
      }
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      const int32_t id = (int32_t)out->size();
      const size_t words = (size_t)id / 64 + 1;
      std::vector<uint64_t> anc(words, 0);
      auto has = [&](const std::vector<uint64_t>& b, int32_t i) {
        return (size_t)i / 64 < b.size() && ((b[(size_t)i / 64] >> (i % 64)) & 1);
      };
      // transitive reduction: drop a candidate that another candidate reaches
      for (int32_t d : cand) {
        bool redundant = false;
        for (int32_t d2 : cand)
          if (d2 != d && has(reach[(size_t)d2], d)) {
            redundant = true;
            break;
          }
        if (!redundant) nd.deps.push_back(d);
        for (size_t w = 0; w < reach[(size_t)d].size(); ++w) anc[w] |= reach[(size_t)d][w];
        anc[(size_t)d / 64] |= uint64_t(1) << (d % 64);
      }
      reach.push_back(std::move(anc));
      out->push_back(std::move(nd));
      acc.emplace_back(rd, wr);
    }
    // the level's kernels touch disjoint data: update the state after all
    for (size_t x = 0; x < acc.size(); ++x) {
      const int32_t id = first + (int32_t)x;
      for (int64_t o : acc[x].first) readers[o].push_back(id);
      for (int64_t o : acc[x].second) {
        last_writer[o] = id;
        readers[o].clear();
      }
    }
  }
}

namespace {

// The contraction levels run one after another, and a level lasts as long as
// its longest work item: the task with the most terms.  An item costs its
// terms' K chunks of 32 plus one per term (its maps) and one (the epilogue).
// A level whose longest item costs at least twice the target -- 2, or the
// mean load of 2,048 work-groups if larger: twice as many as the contraction
// kernel keeps resident (four per compute unit), so that a level's last
// round of items is short (the best of 1,024, 2,048 and 4,096 on MI355X) --
// splits each task costlier than the target into parts of about
// the target, cut at term boundaries (at most 32 parts):
// part 0 keeps the task's output, parts s > 0 write partial slots that a
// fold kernel adds to it after the level (FoldTask).  Slots are reused from
// one level to the next, since the levels run in sequence.
void split_backward(BackPlan* b, int32_t nb) {
  constexpr int32_t kChunk = 32;
  constexpr double kWorkGroups = 2048, kMinCost = 2;
  constexpr int32_t kMaxParts = 32;
  enum { BUF_P = 4 };
  auto term_cost = [&](int32_t t) { return (double)((b->terms[(size_t)t].K + kChunk - 1) / kChunk) + 1.0; };
  auto task_cost = [&](int32_t id) {
    const ConTask& t = b->tasks[(size_t)id];
    double c = 1.0;
    for (int32_t x = t.t_begin; x < t.t_end; ++x) c += term_cost(x);
    return c;
  };
  b->folds.clear();
  b->fold_items.assign(b->level_items.size(), {});
  b->slots = 0;
  for (size_t L = 2; L < b->level_items.size(); ++L) {
    std::vector<int32_t>& items = b->level_items[L];
    double total = 0, longest = 0;
    for (size_t q = 0; q < items.size(); q += 3) {
      const double c = task_cost(items[q]);
      total += c;
      longest = std::max(longest, c);
    }
    const double target = std::max(kMinCost, total / kWorkGroups);
    if (longest < 2 * target) continue;
    std::map<int32_t, std::vector<int32_t>> parts;  // split task -> its part tasks s > 0
    std::map<int32_t, int32_t> fold_of;
    int64_t level_slots = 0;
    for (size_t q = 0; q < items.size(); q += 3) {
      const int32_t id = items[q];
      if (fold_of.count(id) || parts.count(id)) continue;
      const double c = task_cost(id);
      ConTask t = b->tasks[(size_t)id];
      const int32_t nterms = t.t_end - t.t_begin;
      const int32_t np = std::min<int32_t>({kMaxParts, nterms, (int32_t)std::ceil(c / target)});
      if (c <= target || np < 2) {
        parts[id];
        continue;
      }
      // cut points: part k ends at the first term where the running cost
      // reaches (k + 1) / np of the task's term cost
      std::vector<int32_t> cut{t.t_begin};
      double run = 0, tc = c - 1.0;
      for (int32_t x = t.t_begin; x < t.t_end && (int32_t)cut.size() < np; ++x) {
        run += term_cost(x);
        if (run >= tc * (double)cut.size() / np && x + 1 < t.t_end) cut.push_back(x + 1);
      }
      cut.push_back(t.t_end);
      const int32_t nparts = (int32_t)cut.size() - 1;
      if (nparts < 2) {
        parts[id];
        continue;
      }
      b->tasks[(size_t)id].t_end = cut[1];
      const int64_t slot = (int64_t)t.c_rows * nb;
      std::vector<int32_t>& ps = parts[id];
      for (int32_t k = 1; k < nparts; ++k) {
        ConTask pt = t;
        pt.c_off = level_slots + (int64_t)(k - 1) * slot;
        pt.c_buf = BUF_P;
        pt.t_begin = cut[(size_t)k];
        pt.t_end = cut[(size_t)k + 1];
        pt.beta = 0;
        ps.push_back((int32_t)b->tasks.size());
        b->tasks.push_back(pt);
      }
      fold_of[id] = (int32_t)b->folds.size();
      b->folds.push_back(FoldTask{t.c_off, t.c_buf, t.c_rows, t.ncols, t.diag, level_slots, nparts - 1});
      level_slots += (int64_t)(nparts - 1) * slot;
    }
    std::vector<int32_t> out;
    std::vector<int32_t>& fi = b->fold_items[L];
    for (size_t q = 0; q < items.size(); q += 3) {
      const int32_t id = items[q], x = items[q + 1], y = items[q + 2];
      out.insert(out.end(), {id, x, y});
      for (int32_t pid : parts[id]) out.insert(out.end(), {pid, x, y});
      auto f = fold_of.find(id);
      if (f != fold_of.end()) fi.insert(fi.end(), {f->second, x, y});
    }
    items.swap(out);
    b->slots = std::max(b->slots, level_slots);
  }
}

}  // namespace

int build_backward(const Symbolic& s, Plan* p, BackPlan* b, std::string* why) {
  (void)why;
  *b = BackPlan();
  const int32_t nb = s.nb, NT = s.NT;
  const int64_t ntiles = (int64_t)s.tiles.size();
  enum { BUF_L = 0, BUF_Z = 1, BUF_G = 2, BUF_M = 3 };
  enum { NORMAL = 0, TRANS = 1, SYM = 2 };
  std::vector<int64_t> col_first((size_t)NT + 1, 0);
  for (const TileInfo& t : s.tiles) col_first[t.k + 1]++;
  for (int32_t k = 0; k < NT; ++k) col_first[k + 1] += col_first[k];
  auto find_tile = [&](int32_t m, int32_t k) -> int64_t {
    int64_t lo = col_first[k], hi = col_first[k + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if (s.tiles[mid].m < m) lo = mid + 1; else hi = mid;
    }
    return (lo < col_first[k + 1] && s.tiles[lo].m == m) ? lo : -1;
  };
  // per tile: its active rows (local to block m) in the map pool, or -1 when
  // they are 0..n_b-1
  std::vector<int32_t> rows_of((size_t)ntiles, -1);
  for (int64_t t = 0; t < ntiles; ++t) {
    const TileInfo& ti = s.tiles[t];
    if (ti.cnt == nb) continue;
    rows_of[t] = (int32_t)p->maps.size();
    p->maps.insert(p->maps.end(), s.rows.begin() + ti.roff, s.rows.begin() + ti.roff + ti.cnt);
  }
  std::vector<int32_t> pos((size_t)nb);
  auto set_pos = [&](int64_t t) {  // pos[local row] = position in tile t, or -1
    std::fill(pos.begin(), pos.end(), -1);
    const TileInfo& ti = s.tiles[t];
    for (int32_t r = 0; r < ti.cnt; ++r) pos[s.rows[ti.roff + r]] = r;
  };
  auto diag_off = [&](int32_t k) { return (int64_t)k * nb * nb; };
  int32_t nlev = 2;
  b->level_items.resize(2);
  auto add_task = [&](int32_t level, const ConTask& t) {
    if ((int32_t)b->level_items.size() <= level) b->level_items.resize((size_t)level + 1);
    nlev = std::max(nlev, level + 1);
    const int32_t id = (int32_t)b->tasks.size();
    b->tasks.push_back(t);
    const int32_t nbr = (t.c_rows + 63) / 64, nbc = (t.ncols + 63) / 64;
    for (int32_t x = 0; x < nbr; ++x)
      for (int32_t y = 0; y < nbc; ++y) {
        if (t.diag && y > x) continue;
        b->level_items[(size_t)level].push_back(id);
        b->level_items[(size_t)level].push_back(x);
        b->level_items[(size_t)level].push_back(y);
      }
  };
  auto new_task = [&](int64_t c_off, int32_t c_buf, int32_t rows, int32_t cols, int32_t diag,
                      int32_t beta, double alpha) {
    ConTask t{c_off, c_buf, rows, cols, diag, (int32_t)b->terms.size(), 0, beta, alpha};
    return t;
  };
  // level 0: G_k = L_kk^-1 by block columns of 32
  for (int32_t k = 0; k < NT; ++k)
    for (int32_t J = 0; J < nb / 32; ++J) {
      b->trtri_items.push_back(k);
      b->trtri_items.push_back(J);
    }
  // level 1: M_mk = L_mk G_k, and H_k = G_k^T G_k into the diagonal Z tiles
  for (int64_t t = 0; t < ntiles; ++t) {
    const TileInfo& ti = s.tiles[t];
    ConTask task = new_task(p->tile_off[t], BUF_M, ti.cnt, nb, 0, 0, 1.0);
    b->terms.push_back(ConTerm{p->tile_off[t], diag_off(ti.k), BUF_L, NORMAL, -1, -1, BUF_G, -1, nb});
    task.t_end = (int32_t)b->terms.size();
    add_task(1, task);
    b->flops += 2.0 * ti.cnt * nb * nb;
  }
  for (int32_t k = 0; k < NT; ++k) {
    ConTask task = new_task(diag_off(k), BUF_Z, p->diag_h[k], p->diag_h[k], 1, 0, 1.0);
    b->terms.push_back(ConTerm{diag_off(k), diag_off(k), BUF_G, TRANS, -1, -1, BUF_G, -1, nb});
    task.t_end = (int32_t)b->terms.size();
    add_task(1, task);
    b->flops += (double)nb * nb * nb;
  }
  // block columns in descending order; a task's level follows the Z tiles it
  // reads
  std::vector<int32_t> zlev_tile((size_t)ntiles, 1), zlev_diag((size_t)NT, 1);
  for (int32_t k = NT - 1; k >= 0; --k) {
    const int64_t c0 = col_first[k], c1 = col_first[k + 1];
    for (int64_t ti = c0; ti < c1; ++ti) {
      const TileInfo& to = s.tiles[ti];
      const int32_t i = to.m;
      ConTask task = new_task(p->tile_off[ti], BUF_Z, to.cnt, nb, 0, 0, -1.0);
      int32_t lv = 2;
      for (int64_t tm = c0; tm < c1; ++tm) {
        const TileInfo& tb = s.tiles[tm];
        const int32_t m = tb.m;
        // contraction index: the K = cnt(m,k) active rows q of tile (m,k)
        ConTerm c{};
        c.b_buf = BUF_M;
        c.b_off = p->tile_off[tm];
        c.b_qmap = -1;
        c.K = tb.cnt;
        c.a_buf = BUF_Z;
        if (m < i) {  // Z_im = stored tile (i,m): [row of (i,m), q]
          const int64_t tim = find_tile(i, m);
          if (tim < 0) continue;  // no entry of L couples the two blocks
          const TileInfo& ta = s.tiles[tim];
          c.a_off = p->tile_off[tim];
          c.a_mode = NORMAL;
          c.a_qmap = rows_of[tm];
          const bool same = to.cnt == ta.cnt &&
                            std::equal(s.rows.begin() + to.roff,
                                       s.rows.begin() + to.roff + to.cnt, s.rows.begin() + ta.roff);
          if (same) {
            c.a_rmap = -1;
          } else {
            set_pos(tim);
            c.a_rmap = (int32_t)p->maps.size();
            for (int32_t r = 0; r < to.cnt; ++r) p->maps.push_back(pos[s.rows[to.roff + r]]);
          }
          lv = std::max(lv, zlev_tile[tim] + 1);
        } else if (m == i) {  // Z_ii, symmetric, lower triangle stored
          c.a_off = diag_off(i);
          c.a_mode = SYM;
          c.a_rmap = rows_of[ti];
          c.a_qmap = rows_of[tm];
          lv = std::max(lv, zlev_diag[i] + 1);
        } else {  // Z_im = (stored tile (m,i))^T: [row of (m,i) for q, column r]
          const int64_t tmi = find_tile(m, i);
          if (tmi < 0) continue;
          c.a_off = p->tile_off[tmi];
          c.a_mode = TRANS;
          c.a_rmap = rows_of[ti];
          set_pos(tmi);
          c.a_qmap = (int32_t)p->maps.size();
          for (int32_t q = 0; q < tb.cnt; ++q) p->maps.push_back(pos[s.rows[tb.roff + q]]);
          lv = std::max(lv, zlev_tile[tmi] + 1);
        }
        b->terms.push_back(c);
        b->flops += 2.0 * to.cnt * tb.cnt * nb;
      }
      task.t_end = (int32_t)b->terms.size();
      zlev_tile[ti] = lv;
      add_task(lv, task);
    }
    if (c1 == c0) continue;  // Z_kk = H_k
    ConTask dtask = new_task(diag_off(k), BUF_Z, p->diag_h[k], p->diag_h[k], 1, 1, -1.0);
    int32_t lv = 2;
    for (int64_t tm = c0; tm < c1; ++tm) {
      // sum over the active rows q of tile (m,k): M[q, r] Z[q, c]
      b->terms.push_back(ConTerm{p->tile_off[tm], p->tile_off[tm], BUF_M, TRANS, -1, -1, BUF_Z, -1,
                                 s.tiles[tm].cnt});
      lv = std::max(lv, zlev_tile[tm] + 1);
      b->flops += 2.0 * s.tiles[tm].cnt * nb * nb;
    }
    dtask.t_end = (int32_t)b->terms.size();
    zlev_diag[k] = lv;
    add_task(lv, dtask);
  }
  b->level_items.resize((size_t)nlev);
  split_backward(b, nb);
  // input entries on the diagonal: the first entry of each column
  b->diagflag.assign((size_t)s.qnz, 0);
  for (int64_t j = 0; j < s.n; ++j) b->diagflag[(size_t)s.qp[j]] = 1;
  return 0;
}

}  // namespace stc
