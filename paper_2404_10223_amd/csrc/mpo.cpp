// Host construction of the Hamiltonian MPO (complementary-operator form).
//
// H = sum_{pq,s} h_pq a+_ps a_qs + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs.
// Each term is an operator string; sorted by mode (stable, with the fermionic
// sign) its ops sit at sites x_1 <= ... <= x_m.  The channel that carries a
// string across bond b depends on how many of its ops are left of b:
//   0 -> I, all -> H, 1 -> N1(o1), 3 -> C3(o4) (coefficient applied),
//   2 -> N2(o1, o2) while b <= N - b (no coefficient yet), otherwise
//        C2(o3, o4) (coefficient applied, summed over all left pairs).
// The coefficient enters on the first transition into C2, C3 or H, so the
// bond dimension is O(min(b, N-b)^2 + N).  On a site the local operator of a
// transition is the product of the ops placed there (in sorted order) times the
// parity F^(ops placed so far mod 2), the Jordan-Wigner string of the ops still
// to the right.  The channel I runs through the whole chain, so the same sweep
// returns <bra|ket> next to <bra|H|ket>.
#include "mpo.hpp"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <map>
#include <stdexcept>
#include <unordered_map>

namespace tnqe {

namespace {

enum { T_I = 0, T_H = 1, T_N1 = 2, T_N2 = 3, T_C2 = 4, T_C3 = 5 };

struct Op {
  int mode, dag;
};

// 4x4 single-mode operators, [bra][ket], site state k = n_up + 2 n_dn
void single_op(const Op &o, double m[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) m[i][j] = 0.0;
  const bool up = (o.mode % 2) == 0;
  if (up) {            // a+_up: |0> -> |up>, |dn> -> |up dn>
    if (o.dag) { m[1][0] = 1; m[3][2] = 1; } else { m[0][1] = 1; m[2][3] = 1; }
  } else {             // a+_dn: |0> -> |dn>, |up> -> -|up dn>
    if (o.dag) { m[2][0] = 1; m[3][1] = -1; } else { m[0][2] = 1; m[1][3] = -1; }
  }
}

void matmul4(const double a[4][4], const double b[4][4], double c[4][4]) {
  double t[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
      t[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) c[i][j] = t[i][j];
}

struct PatternTable {
  std::vector<OpPattern> list;
  std::map<std::vector<int>, int> index;
  int get(const double m[4][4]) {
    std::vector<int> key;
    OpPattern p;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (m[i][j] != 0.0) {
          if (p.n == 4) throw std::runtime_error("local operator with more than 4 nonzeros");
          key.push_back(i * 16 + j * 4 + (m[i][j] > 0 ? 1 : 2));
          p.kp[p.n] = i;
          p.k[p.n] = j;
          p.f[p.n] = m[i][j];
          ++p.n;
        }
    auto it = index.find(key);
    if (it != index.end()) return it->second;
    const int id = (int)list.size();
    list.push_back(p);
    index.emplace(key, id);
    return id;
  }
};

// Calls f(t, coef_kind, p, q, r, s, ops, m) for every term in a fixed order.
// coef_kind 1: h_pq; 2: 1/2 (pq|rs).
template <class F>
void enumerate_terms(int N, F &&f) {
  int64_t t = 0;
  Op ops[4];
  for (int p = 0; p < N; ++p)
    for (int q = 0; q < N; ++q)
      for (int s = 0; s < 2; ++s) {
        ops[0] = {2 * p + s, 1};
        ops[1] = {2 * q + s, 0};
        f(t++, 1, p, q, 0, 0, ops, 2);
      }
  for (int p = 0; p < N; ++p)
    for (int q = 0; q < N; ++q)
      for (int r = 0; r < N; ++r)
        for (int s_ = 0; s_ < N; ++s_)
          for (int sg = 0; sg < 2; ++sg)
            for (int tu = 0; tu < 2; ++tu) {
              const int mp = 2 * p + sg, mr = 2 * r + tu, ms = 2 * s_ + tu, mq = 2 * q + sg;
              if (mp == mr || ms == mq) {
                ++t;
                continue;
              }
              ops[0] = {mp, 1};
              ops[1] = {mr, 1};
              ops[2] = {ms, 0};
              ops[3] = {mq, 0};
              f(t++, 2, p, q, r, s_, ops, 4);
            }
}

int64_t term_count(int N) { return (int64_t)N * N * 2 + (int64_t)N * N * N * N * 4; }

// smallest coupling block stored dense (TNQE_DENSE_MIN_AREA overrides, for tests)
int64_t dense_min_area() {
  const char *e = std::getenv("TNQE_DENSE_MIN_AREA");
  return e ? std::max<int64_t>(1, std::atoll(e)) : 1024;
}

}  // namespace

void mpo_build_structure(int N, MpoStructure &m) {
  m = MpoStructure();
  m.N = N;
  const int64_t K1 = 4 * N, K2 = K1 * K1;
  auto key_of = [&](int type, int a, int b) -> int64_t {
    if (type == T_N1 || type == T_C3) return type * K2 + a;
    if (type == T_N2 || type == T_C2) return type * K2 + (int64_t)a * K1 + b;
    return type * K2;
  };
  auto normal = [&](int b) { return b <= N - b; };
  // channel keys per bond, in order of first appearance
  std::vector<std::unordered_map<int64_t, int>> chan(N + 1);
  std::vector<std::vector<int64_t>> keys(N + 1);
  auto get_chan = [&](int b, int64_t key) {
    auto it = chan[b].find(key);
    if (it != chan[b].end()) return it->second;
    const int id = (int)keys[b].size();
    keys[b].push_back(key);
    chan[b].emplace(key, id);
    return id;
  };
  for (int b = 0; b <= N; ++b) get_chan(b, key_of(T_I, 0, 0));
  for (int b = 1; b <= N; ++b) get_chan(b, key_of(T_H, 0, 0));

  struct Entry {
    int win, wout, pat, slot;
  };
  std::vector<std::vector<Entry>> entries(N);
  std::vector<std::unordered_map<uint64_t, int>> entry_of(N);
  PatternTable pats;
  const int64_t nterm = term_count(N);
  m.term_slot.assign(nterm, -1);
  m.term_factor.assign(nterm, 0.0);

  auto ekey = [](int win, int wout, int pat) {
    return ((uint64_t)(uint32_t)win << 36) | ((uint64_t)(uint32_t)wout << 12) | (uint64_t)pat;
  };

  enumerate_terms(N, [&](int64_t t, int kind, int, int, int, int, const Op *raw, int mcount) {
    Op o[4];
    for (int i = 0; i < mcount; ++i) o[i] = raw[i];
    double sign = 1.0;
    for (int a = 0; a < mcount; ++a)
      for (int b = 0; b + 1 < mcount - a; ++b)
        if (o[b].mode > o[b + 1].mode) {
          std::swap(o[b], o[b + 1]);
          sign = -sign;
        }
    for (int a = 0; a + 1 < mcount; ++a)
      if (o[a].mode == o[a + 1].mode && o[a].dag == o[a + 1].dag) return;
    int site[4];
    for (int i = 0; i < mcount; ++i) site[i] = o[i].mode / 2;
    auto channel = [&](int j, int b) -> int64_t {
      if (j == 0) return key_of(T_I, 0, 0);
      if (j == mcount) return key_of(T_H, 0, 0);
      if (j == 1) return key_of(T_N1, o[0].mode * 2 + o[0].dag, 0);
      if (j == 2)
        return normal(b) ? key_of(T_N2, o[0].mode * 2 + o[0].dag, o[1].mode * 2 + o[1].dag)
                         : key_of(T_C2, o[2].mode * 2 + o[2].dag, o[3].mode * 2 + o[3].dag);
      return key_of(T_C3, o[3].mode * 2 + o[3].dag, 0);
    };
    bool applied = false;
    for (int x = site[0]; x <= site[mcount - 1]; ++x) {
      int jin = 0, jout = 0;
      for (int i = 0; i < mcount; ++i) {
        jin += site[i] < x;
        jout += site[i] <= x;
      }
      const int64_t kin = channel(jin, x), kout = channel(jout, x + 1);
      if (jin == jout && kin == kout) continue;
      const int win = get_chan(x, kin), wout = get_chan(x + 1, kout);
      double loc[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
      for (int i = 0; i < mcount; ++i)
        if (site[i] == x) {
          double s1[4][4];
          single_op(o[i], s1);
          matmul4(loc, s1, loc);
        }
      if (jout & 1) {
        const double F[4][4] = {{1, 0, 0, 0}, {0, -1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, 1}};
        matmul4(loc, F, loc);
      }
      const int pat = pats.get(loc);
      const int tin = (int)(kin / K2), tout = (int)(kout / K2);
      const bool coef = !applied && (tin == T_I || tin == T_N1 || tin == T_N2) &&
                        (tout == T_C2 || tout == T_C3 || tout == T_H);
      const uint64_t ek = ekey(win, wout, pat);
      auto it = entry_of[x].find(ek);
      if (coef) {
        int slot;
        if (it == entry_of[x].end()) {
          slot = (int)m.nslot++;
          entry_of[x].emplace(ek, (int)entries[x].size());
          entries[x].push_back({win, wout, pat, slot});
        } else {
          slot = entries[x][it->second].slot;
          if (slot < 0) throw std::runtime_error("MPO: structural and coefficient transition collide");
        }
        m.term_slot[t] = slot;
        m.term_factor[t] = sign * (kind == 1 ? 1.0 : 0.5);
        applied = true;
      } else if (it == entry_of[x].end()) {
        entry_of[x].emplace(ek, (int)entries[x].size());
        entries[x].push_back({win, wout, pat, -1});
      } else if (entries[x][it->second].slot >= 0) {
        throw std::runtime_error("MPO: coefficient and structural transition collide");
      }
    }
    if (!applied) throw std::runtime_error("MPO: term without coefficient transition");
  });

  // pass-through of every channel present on both sides of a site
  const double Id[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
  const double Fm[4][4] = {{1, 0, 0, 0}, {0, -1, 0, 0}, {0, 0, -1, 0}, {0, 0, 0, 1}};
  const int patI = pats.get(Id), patF = pats.get(Fm);
  for (int x = 0; x < N; ++x) {
    for (size_t w = 0; w < keys[x].size(); ++w) {
      const int64_t k = keys[x][w];
      auto it = chan[x + 1].find(k);
      if (it == chan[x + 1].end()) continue;
      const int type = (int)(k / K2);
      const int pat = (type == T_N1 || type == T_C3) ? patF : patI;
      const uint64_t ek = ekey((int)w, it->second, pat);
      if (entry_of[x].count(ek)) throw std::runtime_error("MPO: duplicate pass-through");
      entry_of[x].emplace(ek, (int)entries[x].size());
      entries[x].push_back({(int)w, it->second, pat, -1});
    }
  }
  m.patterns = pats.list;

  // classes: shift (bra - ket) of the left operator of each channel
  auto op_shift = [&](int id, int &da, int &db) {
    const int mode = id / 2, dag = id % 2, d = dag ? 1 : -1;
    if (mode % 2 == 0) da += d; else db += d;
  };
  std::vector<std::vector<int>> cls_of(N + 1), loc_of(N + 1);
  m.classes.resize(N + 1);
  for (int b = 0; b <= N; ++b) {
    const size_t n = keys[b].size();
    std::vector<std::array<int, 2>> sh(n);
    for (size_t w = 0; w < n; ++w) {
      const int64_t k = keys[b][w];
      const int type = (int)(k / K2);
      const int64_t id = k % K2;
      int da = 0, db = 0;
      if (type == T_N1) op_shift((int)id, da, db);
      if (type == T_N2) { op_shift((int)(id / K1), da, db); op_shift((int)(id % K1), da, db); }
      if (type == T_C3) { op_shift((int)id, da, db); da = -da; db = -db; }
      if (type == T_C2) {
        op_shift((int)(id / K1), da, db);
        op_shift((int)(id % K1), da, db);
        da = -da;
        db = -db;
      }
      sh[w] = {da, db};
    }
    std::vector<std::array<int, 2>> uniq(sh.begin(), sh.end());
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    // channels of a class ordered by key (type first), so dense groups are contiguous
    std::vector<int> order(n);
    for (size_t w = 0; w < n; ++w) order[w] = (int)w;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return keys[b][x] < keys[b][y]; });
    cls_of[b].assign(n, 0);
    loc_of[b].assign(n, 0);
    m.classes[b].resize(uniq.size());
    for (size_t c = 0; c < uniq.size(); ++c) {
      m.classes[b][c].da = uniq[c][0];
      m.classes[b][c].db = uniq[c][1];
    }
    for (int w : order) {
      const int c = (int)(std::lower_bound(uniq.begin(), uniq.end(), sh[w]) - uniq.begin());
      cls_of[b][w] = c;
      loc_of[b][w] = m.classes[b][c].nw++;
    }
    m.max_bond = std::max<int>(m.max_bond, (int)n);
  }
  m.I_class.assign(N + 1, 0);
  m.I_loc.assign(N + 1, 0);
  for (int b = 0; b <= N; ++b) {
    const int wI = chan[b].at(key_of(T_I, 0, 0));
    m.I_class[b] = cls_of[b][wI];
    m.I_loc[b] = loc_of[b][wI];
  }
  {
    const int wI = chan[N].at(key_of(T_I, 0, 0)), wH = chan[N].at(key_of(T_H, 0, 0));
    if (cls_of[N][wI] != cls_of[N][wH] || m.classes[N].size() != 1 || m.classes[N][0].nw != 2)
      throw std::runtime_error("MPO: unexpected last bond");
    m.final_class = cls_of[N][wI];
    m.final_I = loc_of[N][wI];
    m.final_H = loc_of[N][wH];
  }
  // CSR groups per site
  m.groups.resize(N);
  m.site_nnz.assign(N, 0);
  m.site_nnz_off.assign(N + 1, 0);
  for (int x = 0; x < N; ++x) {
    std::map<std::array<int, 3>, std::vector<std::array<int, 3>>> g;   // -> (row, col, slot)
    for (const Entry &e : entries[x]) {
      const std::array<int, 3> gk = {cls_of[x][e.win], cls_of[x + 1][e.wout], e.pat};
      g[gk].push_back({loc_of[x + 1][e.wout], loc_of[x][e.win], e.slot});
    }
    for (auto &kv : g) {
      MpoGroup grp;
      grp.cin = kv.first[0];
      grp.cout = kv.first[1];
      grp.pattern = kv.first[2];
      auto &v = kv.second;
      std::sort(v.begin(), v.end());
      int rmin = INT32_MAX, rmax = -1, cmin = INT32_MAX, cmax = -1;
      for (auto &e : v) {
        rmin = std::min(rmin, e[0]);
        rmax = std::max(rmax, e[0]);
        cmin = std::min(cmin, e[1]);
        cmax = std::max(cmax, e[1]);
      }
      const int64_t area = (int64_t)(rmax - rmin + 1) * (cmax - cmin + 1);
      if (area >= dense_min_area() && (int64_t)v.size() * 3 >= area) {
        // a coefficient coupling between channel ranges: store it dense
        grp.dense = true;
        grp.r0 = rmin;
        grp.nr = rmax - rmin + 1;
        grp.c0 = cmin;
        grp.nc = cmax - cmin + 1;
        grp.dslot.assign(area, -1);
        for (auto &e : v) grp.dslot[(int64_t)(e[0] - rmin) * grp.nc + (e[1] - cmin)] = e[2] >= 0 ? e[2] : -2;
      } else {
        const int nrow = m.classes[x + 1][grp.cout].nw;
        grp.rowptr.assign(nrow + 1, 0);
        for (auto &e : v) grp.rowptr[e[0] + 1]++;
        for (int r = 0; r < nrow; ++r) grp.rowptr[r + 1] += grp.rowptr[r];
        grp.col.reserve(v.size());
        grp.slot.reserve(v.size());
        for (auto &e : v) {
          grp.col.push_back(e[1]);
          grp.slot.push_back(e[2]);
        }
      }
      grp.val_off = m.site_nnz[x];
      m.site_nnz[x] += grp.nvals();
      m.groups[x].push_back(std::move(grp));
    }
    m.site_nnz_off[x + 1] = m.site_nnz_off[x] + m.site_nnz[x];
  }
}

void mpo_values(const MpoStructure &m, const double *h, const double *g, std::vector<double> &vals,
                std::vector<double> &slotval) {
  const int N = m.N;
  slotval.assign(m.nslot, 0.0);
  const int64_t N2 = (int64_t)N * N, N3 = N2 * N;
  enumerate_terms(N, [&](int64_t t, int kind, int p, int q, int r, int s, const Op *, int) {
    const int slot = m.term_slot[t];
    if (slot < 0) return;
    const double c = kind == 1 ? h[p * N + q] : g[p * N3 + q * N2 + r * N + s];
    slotval[slot] += m.term_factor[t] * c;
  });
  vals.resize(m.site_nnz_off[N]);
  for (int x = 0; x < N; ++x)
    for (const MpoGroup &grp : m.groups[x]) {
      double *o = vals.data() + m.site_nnz_off[x] + grp.val_off;
      if (grp.dense) {
        for (size_t z = 0; z < grp.dslot.size(); ++z) {
          const int sl = grp.dslot[z];
          o[z] = sl >= 0 ? slotval[sl] : (sl == -2 ? 1.0 : 0.0);
        }
      } else {
        for (size_t z = 0; z < grp.slot.size(); ++z) o[z] = grp.slot[z] >= 0 ? slotval[grp.slot[z]] : 1.0;
      }
    }
}

}  // namespace tnqe
