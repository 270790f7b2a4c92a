// ifgf_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU reference for the IFGF evaluation of the discrete
// Helmholtz operator (Bauinger & Bruno, "Massively parallelized interpolated
// factored Green function method", Section 2, eq. (field1)).  It is used by
// the test-suite, by the smoke check and by the CPU baseline of the
// benchmark, never by the library.  It shares no code, header or table with
// the GPU library.
//
// Two functions are provided:
//   * oracle_direct_sum: the O(N^2) definition of eq. (field1) itself,
//       I(x_l) = sum_{m != l} a_m exp(i kappa |x_l - x_m|) / (4 pi |x_l - x_m|).
//   * oracle_ifgf: the IFGF method written out in the order of the paper's
//       Algorithm "IFGF Method" (LevelDEvaluations, then for d = D..3
//       Interpolation(d) and Propagation(d)), plus the level-D neighbour
//       ("LevelDSingularInteractions") direct sum.
//
// Parts the paper leaves to its companion paper, and the readings taken for
// them (all documented in the design notes of the repository):
//   - root cube: bounding cube of the points, centred on the bounding box;
//     box indices are clamped to [0, 2^(d-1) - 1] (points on the max face).
//   - number of levels: D = max(3, 1 + round(log2(H_1 / (leaf_size * lambda)))),
//     or, with an absolute leaf side leaf_abs (the rule that needs no
//     wavelength, used for the Laplace kernel kappa = 0),
//     D = max(3, 1 + round(log2(H_1 / leaf_abs))); an optional cap leaf_max
//     (in wavelengths) then adds levels until H_D <= leaf_max * lambda, which
//     bounds the leaf side of instances whose size rounds badly.
//   - cone coordinates about the box centre x_k: r = |x - x_k|,
//     s = h/r with h = (sqrt 3 / 2) H_d, theta = atan2(sqrt(y1^2+y2^2), y3)
//     in [0, pi], phi = atan2(y2, y1) mapped to [0, 2 pi); s in (0, eta] with
//     eta = sqrt(3)/3.
//   - cone grid: (n_s, n_theta, n_phi) at level D, doubled per dimension for
//     each level up (kappa > 0); for kappa = 0 the analytic factor is
//     scale-free in (s, theta, phi), so the same grid serves every level;
//     cone index gamma = (i_s n_theta + i_theta) n_phi + i_phi
//     ("radial first, then elevation, finally azimuth").
//   - interpolation: tensor-product Chebyshev interpolation at first-kind
//     Chebyshev nodes, P = P_s * P_ang * P_ang points per cone; interpolants are
//     held as Chebyshev coefficients (the "P coefficients" of the paper).
//   - relevant cones (eq. relevantconesegments): a cone is relevant if it
//     contains a cousin point, or an interpolation node of a relevant cone of
//     the parent box (a point-based form of the region intersection rule).
//
// Parity status: the direct sum is pinned by closed forms and invariants in
// the test-suite; the IFGF oracle is pinned by its "exact" mode (interpolant
// evaluations replaced by exact child sums, reproducing the direct sum), by
// exact reproduction of tensor polynomials, by convergence in P and by its
// error against the direct sum.  Its values at the default parameters are
// otherwise "parity unpinned": the paper prints no worked example.

#include <omp.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <unordered_set>
#include <vector>

typedef std::complex<double> cplx;

static const double PI = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Direct sum, eq. (field1).
// ---------------------------------------------------------------------------

// Compensated (Kahan) accumulation of one complex sum.
struct KahanC {
  double sr = 0, cr = 0, si = 0, ci = 0;
  void add(double xr, double xi) {
    double y = xr - cr;
    double t = sr + y;
    cr = (t - sr) - y;
    sr = t;
    y = xi - ci;
    t = si + y;
    ci = (t - si) - y;
    si = t;
  }
};

// Green function G(x,y) = exp(i kappa r) / (4 pi r), r = |x - y|.
static inline cplx green(double r, double kappa) {
  return std::exp(cplx(0.0, kappa * r)) / (4.0 * PI * r);
}

extern "C" int oracle_direct_sum(const double* pts, int64_t n,
                                 const double* dens, double kappa,
                                 const int64_t* targets, int64_t m,
                                 double* out) {
  if (n < 1 || m < 0 || kappa < 0) return 1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < m; ++t) {
    int64_t l = targets[t];
    KahanC acc;
    for (int64_t j = 0; j < n; ++j) {
      if (j == l) continue;
      double dx = pts[3 * l] - pts[3 * j];
      double dy = pts[3 * l + 1] - pts[3 * j + 1];
      double dz = pts[3 * l + 2] - pts[3 * j + 2];
      double r = std::sqrt(dx * dx + dy * dy + dz * dz);
      cplx v = cplx(dens[2 * j], dens[2 * j + 1]) * green(r, kappa);
      acc.add(v.real(), v.imag());
    }
    out[2 * t] = acc.sr;
    out[2 * t + 1] = acc.si;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// IFGF.
// ---------------------------------------------------------------------------

struct Box {
  int64_t first = 0, count = 0;  // points [first, first+count) in sorted order
  int64_t k[3] = {0, 0, 0};      // multi-index in the level grid
  double c[3] = {0, 0, 0};       // box centre x_k^d
};

struct Level {
  int d = 0;
  double H = 0, h = 0;                      // side and half diagonal
  int ns = 0, nt = 0, np = 0;               // cone grid at this level
  double ds = 0, dt = 0, dp = 0;            // cone widths in s, theta, phi
  std::vector<Box> boxes;                   // relevant boxes, Morton order
  std::unordered_map<uint64_t, int64_t> by_key;  // Morton key -> box index
  // Relevant cones: per box a hash map gamma -> offset into `coef`
  // (units of P coefficients), as in the paper's per-box hash maps.
  std::vector<std::unordered_map<int64_t, int64_t>> cone_offset;
  std::vector<std::pair<int64_t, int64_t>> cones;  // (box, gamma) per offset
  std::vector<cplx> coef;                           // Chebyshev coefficients
};

struct Options {
  int p_s, p_ang;
  int ns, nt, np;     // leaf-level cone grid
  int levels;         // 0: automatic D
  int mode;           // 0: interpolated IFGF, 1: exact evaluations
  int stages;         // bit 0: near field, bit 1: far field (levels D..3)
  int grid_rule = 0;  // 0: doubles per level up if kappa > 0, else constant;
                      // 1: always doubles; 2: constant
  double leaf_max = 0;  // cap on the leaf side in wavelengths (0: none)
  double leaf_abs = 0;  // leaf side in length units (0: use leaf_size)
};

struct Oracle {
  int64_t n = 0;
  const double* x_user = nullptr;
  const double* a_user = nullptr;
  double kappa = 0;
  Options o{};
  int D = 0;
  double H1 = 0, corner[3] = {0, 0, 0};
  double setup_seconds = 0, eval_seconds = 0;  // wall times of run()
  std::vector<int64_t> order;      // sorted position -> user index
  std::vector<double> X[3];        // sorted coordinates (SoA)
  std::vector<cplx> A;             // sorted densities
  std::vector<Level> lev;          // lev[d], d = 1..D
  std::vector<double> t_s, t_a;    // Chebyshev nodes on [-1,1]
  int P = 0;
  bool failed = false;             // a cone lookup missed (relevance bug)

  // ---- octree -------------------------------------------------------------

  static uint64_t morton(const int64_t k[3], int bits) {
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b) {
      key = (key << 3) | (uint64_t(((k[0] >> b) & 1)) << 2) |
            (uint64_t(((k[1] >> b) & 1)) << 1) | uint64_t((k[2] >> b) & 1);
    }
    return key;
  }

  void build_tree(double leaf_size) {
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = hi[a] = x_user[a];
      for (int64_t i = 0; i < n; ++i) {
        lo[a] = std::min(lo[a], x_user[3 * i + a]);
        hi[a] = std::max(hi[a], x_user[3 * i + a]);
      }
    }
    H1 = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    for (int a = 0; a < 3; ++a) corner[a] = 0.5 * (lo[a] + hi[a]) - 0.5 * H1;
    if (o.levels > 0) {
      D = o.levels;
    } else if (o.leaf_abs > 0) {
      D = std::max(3, 1 + (int)std::llround(std::log2(H1 / o.leaf_abs)));
    } else {
      double lambda = 2.0 * PI / kappa;
      D = std::max(3, 1 + (int)std::llround(std::log2(H1 / (leaf_size * lambda))));
    }
    // Leaf-side cap: one more level while the leaf is wider than
    // leaf_max wavelengths.
    if (o.levels == 0 && o.leaf_max > 0 && kappa > 0) {
      double lambda = 2.0 * PI / kappa;
      while (D < 21 && std::ldexp(H1, -(D - 1)) > o.leaf_max * lambda) ++D;
    }
    lev.assign(D + 1, Level());
    double HD = std::ldexp(H1, -(D - 1));
    int64_t nbox = int64_t(1) << (D - 1);
    // Leaf multi-index of each point: floor((x - corner) / H_D), clamped.
    std::vector<std::array<int64_t, 3>> kk(n);
    std::vector<uint64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
      for (int a = 0; a < 3; ++a) {
        int64_t k = (int64_t)std::floor((x_user[3 * i + a] - corner[a]) / HD);
        kk[i][a] = std::min(std::max(k, int64_t(0)), nbox - 1);
      }
      key[i] = morton(kk[i].data(), D - 1);
    }
    order.resize(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int64_t p, int64_t q) {
      return key[p] != key[q] ? key[p] < key[q] : p < q;
    });
    for (int a = 0; a < 3; ++a) {
      X[a].resize(n);
      for (int64_t i = 0; i < n; ++i) X[a][i] = x_user[3 * order[i] + a];
    }
    A.resize(n);
    for (int64_t i = 0; i < n; ++i)
      A[i] = cplx(a_user[2 * order[i]], a_user[2 * order[i] + 1]);
    // Boxes of every level: runs of equal ancestor keys in the sorted order.
    for (int d = 1; d <= D; ++d) {
      Level& L = lev[d];
      L.d = d;
      L.H = std::ldexp(H1, -(d - 1));
      L.h = 0.5 * std::sqrt(3.0) * L.H;
      int shift = 3 * (D - d);
      for (int64_t i = 0; i < n; ++i) {
        uint64_t kd = key[order[i]] >> shift;
        bool start = (i == 0) || ((key[order[i - 1]] >> shift) != kd);
        if (start) {
          Box b;
          b.first = i;
          for (int a = 0; a < 3; ++a) {
            b.k[a] = kk[order[i]][a] >> (D - d);
            b.c[a] = corner[a] + (double(b.k[a]) + 0.5) * L.H;
          }
          L.by_key[kd] = (int64_t)L.boxes.size();
          L.boxes.push_back(b);
        }
        L.boxes.back().count += 1;
      }
    }
  }

  // Relevant box at level d with multi-index k, or -1.
  int64_t find_box(int d, const int64_t k[3]) const {
    int64_t nb = int64_t(1) << (d - 1);
    for (int a = 0; a < 3; ++a)
      if (k[a] < 0 || k[a] >= nb) return -1;
    auto it = lev[d].by_key.find(morton(k, d - 1));
    return it == lev[d].by_key.end() ? -1 : it->second;
  }

  // Neighbours N B (eq. defneighboursandcousins): relevant boxes with
  // ||j - k||_inf <= 1, the box itself included.
  std::vector<int64_t> neighbours(int d, int64_t b) const {
    std::vector<int64_t> out;
    const Box& B = lev[d].boxes[b];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t k[3] = {B.k[0] + dx, B.k[1] + dy, B.k[2] + dz};
          int64_t j = find_box(d, k);
          if (j >= 0) out.push_back(j);
        }
    return out;
  }

  int64_t parent(int d, int64_t b) const {
    const Box& B = lev[d].boxes[b];
    int64_t k[3] = {B.k[0] >> 1, B.k[1] >> 1, B.k[2] >> 1};
    return find_box(d - 1, k);
  }

  // Relevant children of box b at level d (boxes of level d+1).
  std::vector<int64_t> children(int d, int64_t b) const {
    std::vector<int64_t> out;
    const Box& B = lev[d].boxes[b];
    for (int o = 0; o < 8; ++o) {
      int64_t k[3] = {2 * B.k[0] + ((o >> 2) & 1), 2 * B.k[1] + ((o >> 1) & 1),
                      2 * B.k[2] + (o & 1)};
      int64_t j = find_box(d + 1, k);
      if (j >= 0) out.push_back(j);
    }
    return out;
  }

  // Cousins M B: relevant non-neighbours whose parent neighbours P B.
  std::vector<int64_t> cousins(int d, int64_t b) const {
    std::vector<int64_t> out;
    const Box& B = lev[d].boxes[b];
    for (int64_t pn : neighbours(d - 1, parent(d, b))) {
      for (int64_t c : children(d - 1, pn)) {
        const Box& C = lev[d].boxes[c];
        int64_t dist = 0;
        for (int a = 0; a < 3; ++a)
          dist = std::max<int64_t>(dist, std::llabs(C.k[a] - B.k[a]));
        if (dist > 1) out.push_back(c);
      }
    }
    return out;
  }

  // ---- cone segments ------------------------------------------------------

  struct ConePos {
    int64_t gamma;
    double u[3];  // local coordinates in [-1, 1]^3
  };

  // Spherical coordinates (s, theta, phi) of y = x - x_k, and the cone
  // containing them with local coordinates.
  ConePos locate(const Level& L, const double y[3]) const {
    double r = std::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double s = L.h / r;
    double th = std::atan2(std::sqrt(y[0] * y[0] + y[1] * y[1]), y[2]);
    double ph = std::atan2(y[1], y[0]);
    if (ph < 0) ph += 2.0 * PI;
    double q[3] = {s / L.ds, th / L.dt, ph / L.dp};
    int nn[3] = {L.ns, L.nt, L.np};
    int64_t idx[3];
    ConePos cp;
    for (int a = 0; a < 3; ++a) {
      int64_t i = (int64_t)std::floor(q[a]);
      i = std::min<int64_t>(std::max<int64_t>(i, 0), nn[a] - 1);
      idx[a] = i;
      cp.u[a] = 2.0 * (q[a] - double(i)) - 1.0;
    }
    cp.gamma = (idx[0] * L.nt + idx[1]) * L.np + idx[2];
    return cp;
  }

  // Cartesian position of interpolation node (ia, ib, ic) of cone gamma of
  // box b: x_k + (h/s) (sin th cos ph, sin th sin ph, cos th).
  void node(const Level& L, int64_t b, int64_t gamma, int ia, int ib, int ic,
            double x[3]) const {
    int64_t is = gamma / (int64_t(L.nt) * L.np);
    int64_t it = (gamma / L.np) % L.nt;
    int64_t ip = gamma % L.np;
    double s = L.ds * (double(is) + 0.5 * (t_s[ia] + 1.0));
    double th = L.dt * (double(it) + 0.5 * (t_a[ib] + 1.0));
    double ph = L.dp * (double(ip) + 0.5 * (t_a[ic] + 1.0));
    double r = L.h / s;
    const Box& B = L.boxes[b];
    x[0] = B.c[0] + r * std::sin(th) * std::cos(ph);
    x[1] = B.c[1] + r * std::sin(th) * std::sin(ph);
    x[2] = B.c[2] + r * std::cos(th);
  }

  void mark(Level& L, int64_t b, std::unordered_set<int64_t>& s,
            const double x[3]) const {
    const Box& B = L.boxes[b];
    double y[3] = {x[0] - B.c[0], x[1] - B.c[1], x[2] - B.c[2]};
    s.insert(locate(L, y).gamma);
  }

  // Relevant cone segments, eq. (relevantconesegments): empty for d = 1, 2;
  // for d >= 3 the cones holding a cousin point or a node of a relevant cone
  // of the parent box.  Computed top-down, d = 3..D.
  void build_cones() {
    const double eta = std::sqrt(3.0) / 3.0;
    for (int d = 3; d <= D; ++d) {
      Level& L = lev[d];
      // Cone grid of level d: the leaf grid, doubled per dimension for each
      // level up when it follows the wavelength.
      const bool doubling = o.grid_rule == 1 || (o.grid_rule == 0 && kappa > 0);
      int f = doubling ? 1 << (D - d) : 1;
      L.ns = o.ns * f;
      L.nt = o.nt * f;
      L.np = o.np * f;
      L.ds = eta / L.ns;
      L.dt = PI / L.nt;
      L.dp = 2.0 * PI / L.np;
      int64_t nb = (int64_t)L.boxes.size();
      std::vector<std::unordered_set<int64_t>> rel(nb);
#pragma omp parallel for schedule(dynamic, 4)
      for (int64_t b = 0; b < nb; ++b) {
        for (int64_t c : cousins(d, b)) {
          const Box& C = L.boxes[c];
          for (int64_t i = C.first; i < C.first + C.count; ++i) {
            double x[3] = {X[0][i], X[1][i], X[2][i]};
            mark(L, b, rel[b], x);
          }
        }
        if (d > 3) {
          const Level& Lp = lev[d - 1];
          int64_t pb = parent(d, b);
          for (auto& kv : Lp.cone_offset[pb]) {
            for (int ia = 0; ia < o.p_s; ++ia)
              for (int ib = 0; ib < o.p_ang; ++ib)
                for (int ic = 0; ic < o.p_ang; ++ic) {
                  double x[3];
                  node(Lp, pb, kv.first, ia, ib, ic, x);
                  mark(L, b, rel[b], x);
                }
          }
        }
      }
      L.cone_offset.assign(nb, {});
      for (int64_t b = 0; b < nb; ++b) {
        std::vector<int64_t> g(rel[b].begin(), rel[b].end());
        std::sort(g.begin(), g.end());
        for (int64_t gamma : g) {
          L.cone_offset[b][gamma] = (int64_t)L.cones.size();
          L.cones.push_back({b, gamma});
        }
      }
      L.coef.assign(L.cones.size() * P, cplx(0, 0));
    }
  }

  // ---- interpolation ------------------------------------------------------

  // Chebyshev polynomials T_0..T_{n-1} at u (three-term recurrence).
  static void cheb_T(int n, double u, double* T) {
    T[0] = 1.0;
    if (n > 1) T[1] = u;
    for (int k = 2; k < n; ++k) T[k] = 2.0 * u * T[k - 1] - T[k - 2];
  }

  // "Generate interpolant": Chebyshev coefficients of the tensor-product
  // interpolant from values at the first-kind nodes,
  //   c_k = (2 - delta_k0)/n * sum_j f(t_j) cos(k (2j+1) pi / (2n)),
  // applied along each of the three dimensions.
  void values_to_coef(const cplx* v, cplx* c) const {
    int ps = o.p_s, pa = o.p_ang;
    std::vector<cplx> w1(P), w2(P);
    auto T = [](int k, int j, int n) {
      return std::cos(double(k) * (2.0 * j + 1.0) * PI / (2.0 * n));
    };
    // phi (last index)
    for (int a = 0; a < ps; ++a)
      for (int b = 0; b < pa; ++b)
        for (int k = 0; k < pa; ++k) {
          cplx s = 0;
          for (int j = 0; j < pa; ++j) s += v[(a * pa + b) * pa + j] * T(k, j, pa);
          w1[(a * pa + b) * pa + k] = s * ((k == 0 ? 1.0 : 2.0) / pa);
        }
    // theta
    for (int a = 0; a < ps; ++a)
      for (int k = 0; k < pa; ++k)
        for (int c3 = 0; c3 < pa; ++c3) {
          cplx s = 0;
          for (int j = 0; j < pa; ++j) s += w1[(a * pa + j) * pa + c3] * T(k, j, pa);
          w2[(a * pa + k) * pa + c3] = s * ((k == 0 ? 1.0 : 2.0) / pa);
        }
    // s
    for (int k = 0; k < ps; ++k)
      for (int b = 0; b < pa; ++b)
        for (int c3 = 0; c3 < pa; ++c3) {
          cplx s = 0;
          for (int j = 0; j < ps; ++j) s += w2[(j * pa + b) * pa + c3] * T(k, j, ps);
          c[(k * pa + b) * pa + c3] = s * ((k == 0 ? 1.0 : 2.0) / ps);
        }
  }

  // Evaluate the interpolant I_P C (coefficients c) at local coordinates u.
  cplx eval_coef(const cplx* c, const double u[3]) const {
    double Ts[16], Tt[16], Tp[16];
    cheb_T(o.p_s, u[0], Ts);
    cheb_T(o.p_ang, u[1], Tt);
    cheb_T(o.p_ang, u[2], Tp);
    cplx s = 0;
    for (int a = 0; a < o.p_s; ++a)
      for (int b = 0; b < o.p_ang; ++b)
        for (int k = 0; k < o.p_ang; ++k)
          s += c[(a * o.p_ang + b) * o.p_ang + k] * (Ts[a] * Tt[b] * Tp[k]);
    return s;
  }

  // F_k^d(x) of eq. (fieldperbox): sum over the points of box b of
  // a(x') g_k(x, x'), g_k(x,x') = G(x,x')/G(x,x_k)
  //                             = (|x-x_k|/|x-x'|) exp(i kappa (|x-x'| - |x-x_k|)).
  cplx field_exact(int d, int64_t b, const double x[3]) const {
    const Box& B = lev[d].boxes[b];
    double rk = std::sqrt((x[0] - B.c[0]) * (x[0] - B.c[0]) +
                          (x[1] - B.c[1]) * (x[1] - B.c[1]) +
                          (x[2] - B.c[2]) * (x[2] - B.c[2]));
    cplx s = 0;
    for (int64_t i = B.first; i < B.first + B.count; ++i) {
      double dx = x[0] - X[0][i], dy = x[1] - X[1][i], dz = x[2] - X[2][i];
      double r = std::sqrt(dx * dx + dy * dy + dz * dz);
      s += A[i] * (rk / r) * std::exp(cplx(0.0, kappa * (r - rk)));
    }
    return s;
  }

  // Value of the level-d interpolant of box b at x (x must lie in one of its
  // relevant cones).  In exact mode the interpolant is replaced by the exact
  // sum over the relevant children, each weighted by G(x,x_child)/G(x,x_k) as
  // in Propagation, down to the exact leaf field.
  cplx eval_box(int d, int64_t b, const double x[3]) {
    const Level& L = lev[d];
    const Box& B = L.boxes[b];
    double y[3] = {x[0] - B.c[0], x[1] - B.c[1], x[2] - B.c[2]};
    ConePos cp = locate(L, y);
    auto it = L.cone_offset[b].find(cp.gamma);
    if (it == L.cone_offset[b].end()) {
      failed = true;
      return 0;
    }
    if (o.mode == 0) return eval_coef(&L.coef[it->second * P], cp.u);
    if (d == D) return field_exact(d, b, x);
    double rj = std::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    cplx s = 0;
    for (int64_t c : children(d, b)) {
      const Box& C = lev[d + 1].boxes[c];
      double rk = std::sqrt((x[0] - C.c[0]) * (x[0] - C.c[0]) +
                            (x[1] - C.c[1]) * (x[1] - C.c[1]) +
                            (x[2] - C.c[2]) * (x[2] - C.c[2]));
      s += eval_box(d + 1, c, x) * (rj / rk) * std::exp(cplx(0.0, kappa * (rk - rj)));
    }
    return s;
  }

  // ---- the algorithm ------------------------------------------------------

  // LevelDEvaluations: F_k^D at the nodes of every relevant leaf cone, then
  // generate the interpolants.
  void level_d_evaluations() {
    Level& L = lev[D];
    int64_t nc = (int64_t)L.cones.size();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      std::vector<cplx> val(P);
      int64_t b = L.cones[c].first, gamma = L.cones[c].second;
      for (int ia = 0; ia < o.p_s; ++ia)
        for (int ib = 0; ib < o.p_ang; ++ib)
          for (int ic = 0; ic < o.p_ang; ++ic) {
            double x[3];
            node(L, b, gamma, ia, ib, ic, x);
            val[(ia * o.p_ang + ib) * o.p_ang + ic] = field_exact(D, b, x);
          }
      values_to_coef(val.data(), &L.coef[c * P]);
    }
  }

  // Interpolation(d), in the per-target form of the parallel algorithm:
  // for each point x and each cousin box B_k of its level-d box, add
  // I_P C_{k;gamma}(x) * G(x, x_k).
  void interpolation(int d, std::vector<cplx>& out) {
    const Level& L = lev[d];
    int64_t nb = (int64_t)L.boxes.size();
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < nb; ++b) {
      std::vector<int64_t> cs = cousins(d, b);
      const Box& B = L.boxes[b];
      for (int64_t i = B.first; i < B.first + B.count; ++i) {
        double x[3] = {X[0][i], X[1][i], X[2][i]};
        cplx s = 0;
        for (int64_t k : cs) {
          const Box& K = L.boxes[k];
          double r = std::sqrt((x[0] - K.c[0]) * (x[0] - K.c[0]) +
                               (x[1] - K.c[1]) * (x[1] - K.c[1]) +
                               (x[2] - K.c[2]) * (x[2] - K.c[2]));
          s += eval_box(d, k, x) * green(r, kappa);
        }
        out[i] += s;
      }
    }
  }

  // Propagation(d), in the per-parent-cone form of the parallel algorithm:
  // for each relevant cone of level d-1 and each of its nodes x, add over the
  // relevant children B_k of its box I_P C_{k;alpha}(x) G(x,x_k)/G(x,x_j);
  // then generate the level d-1 interpolants.
  void propagation(int d) {
    Level& Lp = lev[d - 1];
    int64_t nc = (int64_t)Lp.cones.size();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < nc; ++c) {
      std::vector<cplx> val(P, cplx(0, 0));
      int64_t j = Lp.cones[c].first, gamma = Lp.cones[c].second;
      const Box& J = Lp.boxes[j];
      std::vector<int64_t> ch = children(d - 1, j);
      for (int ia = 0; ia < o.p_s; ++ia)
        for (int ib = 0; ib < o.p_ang; ++ib)
          for (int ic = 0; ic < o.p_ang; ++ic) {
            double x[3];
            node(Lp, j, gamma, ia, ib, ic, x);
            double rj = std::sqrt((x[0] - J.c[0]) * (x[0] - J.c[0]) +
                                  (x[1] - J.c[1]) * (x[1] - J.c[1]) +
                                  (x[2] - J.c[2]) * (x[2] - J.c[2]));
            cplx s = 0;
            for (int64_t k : ch) {
              const Box& K = lev[d].boxes[k];
              double rk = std::sqrt((x[0] - K.c[0]) * (x[0] - K.c[0]) +
                                    (x[1] - K.c[1]) * (x[1] - K.c[1]) +
                                    (x[2] - K.c[2]) * (x[2] - K.c[2]));
              s += eval_box(d, k, x) * (rj / rk) *
                   std::exp(cplx(0.0, kappa * (rk - rj)));
            }
            val[(ia * o.p_ang + ib) * o.p_ang + ic] = s;
          }
      values_to_coef(val.data(), &Lp.coef[c * P]);
    }
  }

  // LevelDSingularInteractions: direct sum over the neighbour points U B^D,
  // the target itself excluded.
  void near_field(std::vector<cplx>& out) {
    const Level& L = lev[D];
    int64_t nb = (int64_t)L.boxes.size();
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < nb; ++b) {
      std::vector<int64_t> nbr = neighbours(D, b);
      const Box& B = L.boxes[b];
      for (int64_t i = B.first; i < B.first + B.count; ++i) {
        cplx s = 0;
        for (int64_t j : nbr) {
          const Box& J = L.boxes[j];
          for (int64_t m = J.first; m < J.first + J.count; ++m) {
            if (m == i) continue;
            double dx = X[0][i] - X[0][m], dy = X[1][i] - X[1][m],
                   dz = X[2][i] - X[2][m];
            s += A[m] * green(std::sqrt(dx * dx + dy * dy + dz * dz), kappa);
          }
        }
        out[i] += s;
      }
    }
  }

  int run(double leaf_size, double* out_user) {
    P = o.p_s * o.p_ang * o.p_ang;
    t_s.resize(o.p_s);
    t_a.resize(o.p_ang);
    for (int j = 0; j < o.p_s; ++j) t_s[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * o.p_s));
    for (int j = 0; j < o.p_ang; ++j) t_a[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * o.p_ang));
    auto t0 = std::chrono::steady_clock::now();
    build_tree(leaf_size);
    build_cones();
    auto t1 = std::chrono::steady_clock::now();
    setup_seconds = std::chrono::duration<double>(t1 - t0).count();
    std::vector<cplx> out(n, cplx(0, 0));
    if (o.stages & 1) near_field(out);
    if (o.stages & 2) {
      if (o.mode == 0) level_d_evaluations();
      for (int d = D; d >= 3; --d) {
        interpolation(d, out);
        if (d > 3 && o.mode == 0) propagation(d);
      }
    }
    eval_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    if (failed) return 3;
    for (int64_t i = 0; i < n; ++i) {
      out_user[2 * order[i]] = out[i].real();
      out_user[2 * order[i] + 1] = out[i].imag();
    }
    return 0;
  }
};

// opts: {p_s, p_ang, ns, nt, np, levels, mode, stages, grid_rule}
// dopts: {leaf_max, leaf_abs} (may be null: both 0)
// info (optional, length >= 2 + 2*32 + 2): [D, H1, then per level d=1..D the
// number of relevant boxes and relevant cones, then at [66] the wall time of
// the set-up (tree, lists, relevant cones) and at [67] that of the
// evaluation (near field, leaf evaluations, interpolation, propagation), in
// seconds].
// Options of the oracle from the flat arrays of the C interface; false when
// they do not define a level rule (kappa = 0 needs levels or leaf_abs).
static bool read_options(Options& o, const int* opts, const double* dopts,
                         double kappa, double leaf_size) {
  o = Options{opts[0], opts[1], opts[2], opts[3], opts[4], opts[5], opts[6], opts[7]};
  o.grid_rule = opts[8];
  if (dopts) {
    o.leaf_max = dopts[0];
    o.leaf_abs = dopts[1];
  }
  if (!(kappa >= 0) || !std::isfinite(kappa)) return false;
  if (o.grid_rule < 0 || o.grid_rule > 2 || !(o.leaf_max >= 0) || !(o.leaf_abs >= 0)) return false;
  if (o.levels == 0 && o.leaf_abs == 0 && !(kappa > 0 && leaf_size > 0)) return false;
  return true;
}

extern "C" int oracle_ifgf(const double* pts, int64_t n, const double* dens,
                           double kappa, double leaf_size, const int* opts,
                           const double* dopts, double* out, double* info) {
  if (n < 2) return 1;
  Oracle O;
  O.n = n;
  O.x_user = pts;
  O.a_user = dens;
  O.kappa = kappa;
  if (!read_options(O.o, opts, dopts, kappa, leaf_size)) return 1;
  if (O.o.p_s < 1 || O.o.p_ang < 1 || O.o.p_s > 16 || O.o.p_ang > 16) return 1;
  int rc = O.run(leaf_size, out);
  if (info) {
    info[0] = O.D;
    info[1] = O.H1;
    for (int d = 1; d <= O.D && d <= 32; ++d) {
      info[2 * d] = (double)O.lev[d].boxes.size();
      info[2 * d + 1] = (double)O.lev[d].cones.size();
    }
    info[66] = O.setup_seconds;
    info[67] = O.eval_seconds;
  }
  return rc;
}

// OpenMP threads the oracle's parallel loops use.
extern "C" int oracle_threads() { return omp_get_max_threads(); }

// Interaction count per target: points in U B^D(x) (self included) plus the
// points of every cousin box at levels D..3.  The paper's partition of the
// sources (near field plus cousins of levels D..3) makes this N for every x.
extern "C" int oracle_partition_counts(const double* pts, int64_t n,
                                       double kappa, double leaf_size,
                                       const int* opts, const double* dopts,
                                       int64_t* counts) {
  if (n < 2) return 1;
  Oracle O;
  O.n = n;
  O.x_user = pts;
  std::vector<double> zero(2 * n, 0.0);
  O.a_user = zero.data();
  O.kappa = kappa;
  if (!read_options(O.o, opts, dopts, kappa, leaf_size)) return 1;
  O.build_tree(leaf_size);
  std::vector<int64_t> cnt(n, 0);
  int D = O.D;
  for (int d = 3; d <= D; ++d) {
    const Level& L = O.lev[d];
    for (int64_t b = 0; b < (int64_t)L.boxes.size(); ++b) {
      int64_t s = 0;
      for (int64_t c : O.cousins(d, b)) s += L.boxes[c].count;
      if (d == D)
        for (int64_t c : O.neighbours(d, b)) s += L.boxes[c].count;
      for (int64_t i = L.boxes[b].first; i < L.boxes[b].first + L.boxes[b].count; ++i)
        cnt[i] += s;
    }
  }
  for (int64_t i = 0; i < n; ++i) counts[O.order[i]] = cnt[i];
  return 0;
}

// The interpolation operator alone, for pins: values of a function at the
// nodes of one cone (ordered (s, theta, phi), phi fastest) -> coefficients
// -> value at local coordinates u.  Used to check exact reproduction of
// tensor polynomials of degree < (p_s, p_ang, p_ang).
extern "C" int oracle_interp_nodes(int p_s, int p_ang, double* t_s, double* t_a) {
  for (int j = 0; j < p_s; ++j) t_s[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * p_s));
  for (int j = 0; j < p_ang; ++j) t_a[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * p_ang));
  return 0;
}

extern "C" int oracle_interp_eval(int p_s, int p_ang, const double* values,
                                  const double* u, int64_t m, double* out) {
  Oracle O;
  O.o.p_s = p_s;
  O.o.p_ang = p_ang;
  O.P = p_s * p_ang * p_ang;
  std::vector<cplx> v(O.P), c(O.P);
  for (int q = 0; q < O.P; ++q) v[q] = cplx(values[2 * q], values[2 * q + 1]);
  O.values_to_coef(v.data(), c.data());
  for (int64_t i = 0; i < m; ++i) {
    cplx r = O.eval_coef(c.data(), &u[3 * i]);
    out[2 * i] = r.real();
    out[2 * i + 1] = r.imag();
  }
  return 0;
}

// Relevant cone segments of level d as sorted keys box * (n_s n_theta n_phi)
// + gamma (boxes numbered in Morton order).  Returns the number of keys
// (writing at most cap of them), or -1 on invalid input.
extern "C" int64_t oracle_cone_keys(const double* pts, int64_t n, double kappa,
                                    double leaf_size, const int* opts,
                                    const double* dopts, int d, uint64_t* out,
                                    int64_t cap) {
  if (n < 2) return -1;
  Oracle O;
  O.n = n;
  O.x_user = pts;
  std::vector<double> zero(2 * n, 0.0);
  O.a_user = zero.data();
  O.kappa = kappa;
  if (!read_options(O.o, opts, dopts, kappa, leaf_size)) return -1;
  O.o.mode = 0;
  O.o.stages = 0;
  O.P = O.o.p_s * O.o.p_ang * O.o.p_ang;
  O.t_s.resize(O.o.p_s);
  O.t_a.resize(O.o.p_ang);
  for (int j = 0; j < O.o.p_s; ++j) O.t_s[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * O.o.p_s));
  for (int j = 0; j < O.o.p_ang; ++j) O.t_a[j] = std::cos((2.0 * j + 1.0) * PI / (2.0 * O.o.p_ang));
  O.build_tree(leaf_size);
  if (d < 3 || d > O.D) return -1;
  O.build_cones();
  const Level& L = O.lev[d];
  uint64_t grid = (uint64_t)L.ns * L.nt * L.np;
  int64_t cnt = (int64_t)L.cones.size();
  for (int64_t i = 0; i < cnt && i < cap; ++i)
    out[i] = (uint64_t)L.cones[i].first * grid + (uint64_t)L.cones[i].second;
  return cnt;
}
