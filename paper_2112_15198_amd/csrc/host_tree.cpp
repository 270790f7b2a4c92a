// host_tree.cpp -- host-side octree, Morton order and interaction lists.
//
// Section 2 of the paper: the cube B^1 containing the points is split
// recursively into half-open boxes of side H_d = H_{d-1}/2; relevant boxes
// contain at least one point; N B = relevant boxes with ||j-k||_inf <= 1
// (the box itself included), M B = relevant children of the parent's
// neighbours that are not neighbours (eq. defneighboursandcousins).
// Section 3.2: points sorted by the Morton key of their level-D box, which
// makes the points of every box contiguous at every level (linear octree).
#include "host_tree.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <thread>

#include "../../include/ifgf.h"

namespace ifgf {

static const double kPi = 3.14159265358979323846;

int default_threads() {
  const char* e = std::getenv("OMP_NUM_THREADS");
  int t = e ? std::atoi(e) : 0;
  if (t <= 0) t = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(t, 64));
}

template <class F>
static void parallel_for(int64_t n, int threads, F f) {
  if (n <= 0) return;
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, n));
  std::atomic<int64_t> next(0);
  int64_t chunk = std::max<int64_t>(1, n / (int64_t(threads) * 32));
  auto work = [&]() {
    for (;;) {
      int64_t b = next.fetch_add(chunk);
      if (b >= n) break;
      int64_t e = std::min(n, b + chunk);
      for (int64_t i = b; i < e; ++i) f(i);
    }
  };
  std::vector<std::thread> ts;
  for (int t = 1; t < threads; ++t) ts.emplace_back(work);
  work();
  for (auto& th : ts) th.join();
}

// Spread the low 21 bits of v so that bit b moves to bit 3b.
static inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

// Morton key: bit interleave with x the most significant bit of each triple.
static inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return (spread3(x) << 2) | (spread3(y) << 1) | spread3(z);
}

int build_instance(const double* pts, int64_t n, double kappa,
                   const LevelRule& rule, InstanceTree& t, std::string& msg) {
  if (n < 2) { msg = "need at least 2 points"; return IFGF_EINVAL; }
  if (n >= (int64_t(1) << 31)) { msg = "N >= 2^31"; return IFGF_EUNSUPPORTED; }
  if (!(kappa >= 0) || !std::isfinite(kappa)) { msg = "kappa must be finite and >= 0"; return IFGF_EINVAL; }
  if (!(rule.leaf_abs >= 0) || !std::isfinite(rule.leaf_abs) || !(rule.leaf_max >= 0) ||
      !std::isfinite(rule.leaf_max)) {
    msg = "leaf_abs and leaf_max must be finite and >= 0";
    return IFGF_EINVAL;
  }
  if (rule.levels == 0 && rule.leaf_abs == 0) {
    if (!(kappa > 0)) { msg = "kappa = 0 needs levels or leaf_abs (no wavelength)"; return IFGF_EINVAL; }
    if (!(rule.leaf_size > 0) || !std::isfinite(rule.leaf_size)) { msg = "leaf_size must be > 0"; return IFGF_EINVAL; }
  }
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) { lo[a] = pts[a]; hi[a] = pts[a]; }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      double v = pts[3 * i + a];
      if (!std::isfinite(v)) { msg = "non-finite coordinate"; return IFGF_EINVAL; }
      lo[a] = std::min(lo[a], v);
      hi[a] = std::max(hi[a], v);
    }
  t.n = n;
  t.kappa = kappa;
  // Root cube B^1: the bounding cube, centred on the bounding box.
  t.H1 = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  if (!(t.H1 > 0)) { msg = "all points coincide"; return IFGF_EDUPLICATE; }
  for (int a = 0; a < 3; ++a) t.corner[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * t.H1;
  if (rule.levels > 0) {
    t.D = rule.levels;
  } else if (rule.leaf_abs > 0) {
    t.D = std::max(3, 1 + (int)std::llround(std::log2(t.H1 / rule.leaf_abs)));
  } else {
    double lambda = 2.0 * kPi / kappa;
    t.D = std::max(3, 1 + (int)std::llround(std::log2(t.H1 / (rule.leaf_size * lambda))));
  }
  // Leaf-side cap (per-instance accuracy control): one more level while the
  // leaf is wider than leaf_max wavelengths.
  if (rule.levels == 0 && rule.leaf_max > 0 && kappa > 0) {
    double lambda = 2.0 * kPi / kappa;
    while (t.D < 21 && std::ldexp(t.H1, -(t.D - 1)) > rule.leaf_max * lambda) ++t.D;
  }
  if (t.D < 3) { msg = "levels must be >= 3"; return IFGF_EINVAL; }
  if (t.D > 21) { msg = "more than 21 levels"; return IFGF_EUNSUPPORTED; }
  const int D = t.D;
  const double HD = std::ldexp(t.H1, -(D - 1));
  const int32_t nside = int32_t(1) << (D - 1);

  // Leaf multi-index floor((x - corner)/H_D), clamped so that points on the
  // max faces fall in the last box, and its Morton key.
  std::vector<int32_t> kk(3 * n);
  std::vector<std::pair<uint64_t, int64_t>> kp(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a) {
      double q = std::floor((pts[3 * i + a] - t.corner[a]) / HD);
      int64_t k = (int64_t)q;
      k = std::min<int64_t>(std::max<int64_t>(k, 0), nside - 1);
      kk[3 * i + a] = (int32_t)k;
    }
    kp[i] = {morton3(kk[3 * i], kk[3 * i + 1], kk[3 * i + 2]), i};
  }
  std::sort(kp.begin(), kp.end());
  t.order.resize(n);
  for (int64_t i = 0; i < n; ++i) t.order[i] = kp[i].second;
  for (int a = 0; a < 3; ++a) {
    t.xs[a].resize(n);
    for (int64_t i = 0; i < n; ++i) t.xs[a][i] = pts[3 * t.order[i] + a];
  }

  // Duplicate points share a leaf box: compare within each leaf run.
  for (int64_t b = 0; b < n;) {
    int64_t e = b;
    while (e < n && kp[e].first == kp[b].first) ++e;
    std::vector<int64_t> idx(t.order.begin() + b, t.order.begin() + e);
    std::sort(idx.begin(), idx.end(), [&](int64_t p, int64_t q) {
      for (int a = 0; a < 3; ++a)
        if (pts[3 * p + a] != pts[3 * q + a]) return pts[3 * p + a] < pts[3 * q + a];
      return p < q;
    });
    for (size_t j = 1; j < idx.size(); ++j)
      if (pts[3 * idx[j]] == pts[3 * idx[j - 1]] &&
          pts[3 * idx[j] + 1] == pts[3 * idx[j - 1] + 1] &&
          pts[3 * idx[j] + 2] == pts[3 * idx[j - 1] + 2]) {
        msg = "duplicate points";
        return IFGF_EDUPLICATE;
      }
    b = e;
  }

  // Level D boxes: runs of equal keys.  Level d-1 boxes: runs of key >> 3
  // over the level-d boxes.
  t.lev.assign(D + 1, TreeLevel());
  {
    TreeLevel& L = t.lev[D];
    for (int64_t i = 0; i < n; ++i) {
      if (i == 0 || kp[i].first != kp[i - 1].first) {
        L.key.push_back(kp[i].first);
        L.first.push_back(i);
        L.count.push_back(0);
        int64_t u = kp[i].second;
        L.k.push_back(kk[3 * u]);
        L.k.push_back(kk[3 * u + 1]);
        L.k.push_back(kk[3 * u + 2]);
      }
      L.count.back() += 1;
    }
  }
  for (int d = D; d >= 2; --d) {
    TreeLevel& C = t.lev[d];
    TreeLevel& Pn = t.lev[d - 1];
    int64_t nb = (int64_t)C.key.size();
    C.parent.assign(nb, -1);
    for (int64_t b = 0; b < nb; ++b) {
      uint64_t pk = C.key[b] >> 3;
      if (Pn.key.empty() || Pn.key.back() != pk) {
        Pn.key.push_back(pk);
        Pn.first.push_back(C.first[b]);
        Pn.count.push_back(0);
        for (int a = 0; a < 3; ++a) Pn.k.push_back(C.k[3 * b + a] >> 1);
      }
      Pn.count.back() += C.count[b];
      C.parent[b] = (int32_t)(Pn.key.size() - 1);
    }
    Pn.child.assign(Pn.key.size() * 8, -1);
    for (int64_t b = 0; b < nb; ++b)
      Pn.child[int64_t(C.parent[b]) * 8 + (C.key[b] & 7)] = (int32_t)b;
  }
  t.lev[1].parent.assign(t.lev[1].key.size(), -1);
  t.lev[D].child.assign(t.lev[D].key.size() * 8, -1);
  return IFGF_OK;
}

static int32_t find_box(const TreeLevel& L, int d, int32_t kx, int32_t ky,
                        int32_t kz) {
  const int32_t nside = int32_t(1) << (d - 1);
  if (kx < 0 || ky < 0 || kz < 0 || kx >= nside || ky >= nside || kz >= nside)
    return -1;
  uint64_t key = morton3(kx, ky, kz);
  auto it = std::lower_bound(L.key.begin(), L.key.end(), key);
  if (it == L.key.end() || *it != key) return -1;
  return (int32_t)(it - L.key.begin());
}

template <class Vec>
static void to_csr(std::vector<Vec>& per, std::vector<int64_t>& begin,
                   std::vector<int32_t>& list) {
  begin.assign(per.size() + 1, 0);
  for (size_t b = 0; b < per.size(); ++b) begin[b + 1] = begin[b] + (int64_t)per[b].size();
  list.resize(begin.back());
  for (size_t b = 0; b < per.size(); ++b)
    std::copy(per[b].begin(), per[b].end(), list.begin() + begin[b]);
  per.clear();
  per.shrink_to_fit();
}

void build_lists(InstanceTree& t, int threads) {
  const int D = t.D;
  // Level-D neighbours, self included.
  {
    const TreeLevel& L = t.lev[D];
    int64_t nb = (int64_t)L.key.size();
    std::vector<std::vector<int32_t>> per(nb);
    parallel_for(nb, threads, [&](int64_t b) {
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int32_t j = find_box(L, D, L.k[3 * b] + dx, L.k[3 * b + 1] + dy,
                                 L.k[3 * b + 2] + dz);
            if (j >= 0) per[b].push_back(j);
          }
    });
    to_csr(per, t.nbr_begin, t.nbr);
  }
  // Cousins at levels 3..D.
  for (int d = 3; d <= D; ++d) {
    TreeLevel& L = t.lev[d];
    const TreeLevel& Pn = t.lev[d - 1];
    int64_t nb = (int64_t)L.key.size();
    std::vector<std::vector<int32_t>> per(nb);
    parallel_for(nb, threads, [&](int64_t b) {
      int32_t p = L.parent[b];
      const int32_t* kb = &L.k[3 * b];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int32_t pn = find_box(Pn, d - 1, Pn.k[3 * p] + dx,
                                  Pn.k[3 * p + 1] + dy, Pn.k[3 * p + 2] + dz);
            if (pn < 0) continue;
            for (int o = 0; o < 8; ++o) {
              int32_t c = Pn.child[int64_t(pn) * 8 + o];
              if (c < 0) continue;
              const int32_t* kc = &L.k[3 * int64_t(c)];
              int32_t dist = std::max(std::abs(kc[0] - kb[0]),
                                      std::max(std::abs(kc[1] - kb[1]),
                                               std::abs(kc[2] - kb[2])));
              if (dist > 1) per[b].push_back(c);
            }
          }
    });
    to_csr(per, L.cous_begin, L.cous);
  }
}

int merge_instances(std::vector<InstanceTree>& trees, Merged& m,
                    std::string& msg) {
  m.n_inst = (int)trees.size();
  m.inst_offset.assign(m.n_inst + 1, 0);
  m.max_D = 0;
  for (int i = 0; i < m.n_inst; ++i) {
    m.inst_offset[i + 1] = m.inst_offset[i] + trees[i].n;
    m.max_D = std::max(m.max_D, trees[i].D);
    trees[i].offset = m.inst_offset[i];
    m.inst_kappa.push_back(trees[i].kappa);
    m.inst_D.push_back(trees[i].D);
  }
  m.n = m.inst_offset.back();
  if (m.n >= (int64_t(1) << 31)) { msg = "N >= 2^31"; return IFGF_EUNSUPPORTED; }
  m.n_steps = m.max_D - 2;
  if (m.n_steps > IFGF_MAX_LEVELS) { msg = "too many levels"; return IFGF_EUNSUPPORTED; }
  m.perm.resize(m.n);
  for (int i = 0; i < m.n_inst; ++i)
    for (int64_t j = 0; j < trees[i].n; ++j)
      m.perm[trees[i].offset + j] = (int32_t)(trees[i].offset + trees[i].order[j]);

  // Per step, the box offset of every instance.
  std::vector<std::vector<int64_t>> boff(m.n_steps, std::vector<int64_t>(m.n_inst + 1, 0));
  for (int l = 0; l < m.n_steps; ++l)
    for (int i = 0; i < m.n_inst; ++i) {
      int d = trees[i].D - l;
      int64_t nb = d >= 3 ? (int64_t)trees[i].lev[d].key.size() : 0;
      boff[l][i + 1] = boff[l][i] + nb;
    }
  m.step.assign(m.n_steps, MergedStep());
  for (int l = 0; l < m.n_steps; ++l) {
    MergedStep& S = m.step[l];
    S.nb = boff[l][m.n_inst];
    S.center.resize(3 * S.nb);
    S.inst.resize(S.nb);
    S.first.resize(S.nb);
    S.count.resize(S.nb);
    S.child.assign(l >= 1 ? 8 * S.nb : 0, -1);
    S.cous_begin.assign(S.nb + 1, 0);
    S.pt_box.assign(m.n, -1);
    S.inst_h.assign(m.n_inst, 0.0);
    S.inst_H.assign(m.n_inst, 0.0);
    int64_t ncous = 0;
    for (int i = 0; i < m.n_inst; ++i) {
      int d = trees[i].D - l;
      if (d >= 3) ncous += (int64_t)trees[i].lev[d].cous.size();
    }
    S.cous.resize(ncous);
    int64_t cpos = 0;
    for (int i = 0; i < m.n_inst; ++i) {
      const InstanceTree& t = trees[i];
      int d = t.D - l;
      if (d < 3) continue;
      const TreeLevel& L = t.lev[d];
      double H = std::ldexp(t.H1, -(d - 1));
      S.inst_H[i] = H;
      S.inst_h[i] = 0.5 * std::sqrt(3.0) * H;
      int64_t o = boff[l][i];
      for (int64_t b = 0; b < (int64_t)L.key.size(); ++b) {
        int64_t g = o + b;
        for (int a = 0; a < 3; ++a)
          S.center[3 * g + a] = t.corner[a] + (double(L.k[3 * b + a]) + 0.5) * H;
        S.inst[g] = i;
        S.first[g] = (int32_t)(t.offset + L.first[b]);
        S.count[g] = L.count[b];
        if (l >= 1)
          for (int c = 0; c < 8; ++c) {
            int32_t ch = L.child[8 * b + c];
            S.child[8 * g + c] = ch < 0 ? -1 : (int32_t)(boff[l - 1][i] + ch);
          }
        for (int64_t j = L.cous_begin[b]; j < L.cous_begin[b + 1]; ++j)
          S.cous[cpos++] = (int32_t)(o + L.cous[j]);
        S.cous_begin[g + 1] = cpos;
        for (int64_t p = S.first[g]; p < S.first[g] + S.count[g]; ++p) S.pt_box[p] = (int32_t)g;
      }
    }
  }
  // Leaf neighbour lists, global.
  m.nbr_begin.assign(m.step[0].nb + 1, 0);
  int64_t tot = 0;
  for (auto& t : trees) tot += (int64_t)t.nbr.size();
  m.nbr.resize(tot);
  int64_t pos = 0;
  m.near_pairs = 0;
  for (int i = 0; i < m.n_inst; ++i) {
    const InstanceTree& t = trees[i];
    int64_t o = boff[0][i];
    const TreeLevel& L = t.lev[t.D];
    for (int64_t b = 0; b < (int64_t)L.key.size(); ++b) {
      int64_t s = 0;
      for (int64_t j = t.nbr_begin[b]; j < t.nbr_begin[b + 1]; ++j) {
        m.nbr[pos++] = (int32_t)(o + t.nbr[j]);
        s += L.count[t.nbr[j]];
      }
      m.nbr_begin[o + b + 1] = pos;
      m.near_pairs += s * L.count[b];
    }
  }
  for (int a = 0; a < 3; ++a) {
    m.xs[a].resize(m.n);
    for (auto& t : trees)
      std::copy(t.xs[a].begin(), t.xs[a].end(), m.xs[a].begin() + t.offset);
  }
  return IFGF_OK;
}

void partition_counts(const Merged& m, int64_t* counts) {
  std::vector<int64_t> cnt(m.n, 0);
  for (int l = 0; l < m.n_steps; ++l) {
    const MergedStep& S = m.step[l];
    for (int64_t b = 0; b < S.nb; ++b) {
      int64_t s = 0;
      for (int64_t j = S.cous_begin[b]; j < S.cous_begin[b + 1]; ++j) s += S.count[S.cous[j]];
      if (l == 0)
        for (int64_t j = m.nbr_begin[b]; j < m.nbr_begin[b + 1]; ++j) s += S.count[m.nbr[j]];
      for (int64_t p = S.first[b]; p < S.first[b] + S.count[b]; ++p) cnt[p] += s;
    }
  }
  for (int64_t p = 0; p < m.n; ++p) counts[m.perm[p]] = cnt[p];
}

}  // namespace ifgf
