// ifgf_kernels.hip -- gfx950 kernels of the IFGF evaluation.
//
// Numerical stages (paper, Section 2 and Algorithms "IFGF Method",
// "Parallel LevelDEvaluations", "Parallel Propagation", "Parallel
// Interpolation"):
//   near_field_kernel    LevelDSingularInteractions: direct sum over the
//                        level-D neighbour points, self excluded.
//   leaf_eval_kernel     LevelDEvaluations: F_k^D (eq. fieldperbox) at the
//                        interpolation nodes of every relevant leaf cone.
//   interp_kernel        Interpolation(d): per target, sum over its cousin
//                        boxes of I_P C(x) * G(x, x_k).
//   prop_*_kernel        Propagation(d): per relevant parent cone node x,
//                        sum over relevant children of I_P C_k(x) *
//                        G(x,x_k)/G(x,x_j).
// Plan-time kernels build the relevant cone segments
// (eq. relevantconesegments) top-down, as open-addressing hash tables keyed
// by (box, cone index) -- the GPU form of the per-box hash maps of
// Section 3.2.2.
//
// Interpolants are stored as values at the tensor Chebyshev (first kind)
// nodes and evaluated with Lagrange weights in product form; this is the same
// polynomial as the coefficient form ("generate interpolant" becomes the
// identity).  Every pass is target-owned: no atomics in the apply.
//
// Precision: T = double (FP64 mode) or float (FP32-mixed mode: values,
// Lagrange weights, contractions and the phase factor's sine and cosine in
// FP32; geometry, the radial cone, the angular cone decisions (side tests)
// and the phase argument kappa*r reduction in FP64; the angular estimates
// and local coordinates of the propagation's cone selection in FP32).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <rocprim/device/device_radix_sort.hpp>

#include "ifgf_device.h"

namespace ifgf {

#define IFGF_NO_CONTRACT _Pragma("clang fp contract(off)")

static constexpr double kPiD = 3.14159265358979323846;
static constexpr double kInv2Pi = 0.15915494309189533577;

// Flat thread index of a launch whose grid is split over x and y (so that
// each dimension stays within the dispatch's 32-bit work-item count).
__device__ __forceinline__ int64_t gtid() {
  return ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ unsigned long long hmix(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

// Slot of (box, gamma) in a level's relevant-cone table, or -1.
__device__ __forceinline__ int cone_lookup(const StepDev& S,
                                           unsigned long long key) {
  if (S.table) return S.table[key];
  unsigned long long h = hmix(key) & S.hmask;
  for (unsigned long long probe = 0; probe <= S.hmask; ++probe) {
    unsigned long long k = S.hkey[h];
    if (k == key) return S.hval[h];
    if (k == kEmptyKey) return -1;
    h = (h + 1) & S.hmask;
  }
  return -1;
}

// Cone coordinates of y = x - x_k about a box centre (FP64, no FMA
// contraction so that host and device round identically):
// r = |y|, s = h/r, theta = atan2(|y_12|, y_3), phi = atan2(y_2, y_1) in
// [0, 2 pi); q = (s/ds, theta/dt, phi/dp).
struct ConeCoord {
  double r;
  double q[3];
};

__device__ __forceinline__ ConeCoord cone_coord(const StepDev& S, double h,
                                                double y0, double y1,
                                                double y2) {
  IFGF_NO_CONTRACT
  ConeCoord c;
  double rho2 = y0 * y0 + y1 * y1;
  c.r = sqrt(rho2 + y2 * y2);
  double s = h / c.r;
  double th = atan2(sqrt(rho2), y2);
  double ph = atan2(y1, y0);
  if (ph < 0) ph += 2.0 * kPiD;
  c.q[0] = s / S.ds;
  c.q[1] = th / S.dt;
  c.q[2] = ph / S.dp;
  return c;
}

__device__ __forceinline__ int cone_index(double q, int n, double& u) {
  IFGF_NO_CONTRACT
  double f = floor(q);
  int i = (int)f;
  if (f < 0) i = 0;
  if (i > n - 1) i = n - 1;
  u = 2.0 * (q - (double)i) - 1.0;
  return i;
}

// Cone selection of the apply: the cone index gamma of y = x - x_k, its local
// coordinates u in [-1, 1]^3 and r = |y| with 1/r.
struct ConeSel {
  int64_t gamma;
  double r, rinv;
};

// atan2(y, x) to about 1.2e-5 rad, as the first guess of a cone index:
// octant reduction and the odd polynomial of Abramowitz and Stegun 4.4.49
// on [0, 1].
__device__ __forceinline__ float atan2_est(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float s = a * a;
  float r = a * (0.9998660f +
                 s * (-0.3302995f + s * (0.1801410f + s * (-0.0851330f + s * 0.0208351f))));
  if (ay > ax) r = 1.57079633f - r;
  if (x < 0.0f) r = 3.14159265f - r;
  return y < 0.0f ? -r : r;
}

// One angle of the FP32-mixed cone selection.  The angle is atan2(Y, X),
// est an estimate of it (>= 0) and bnd the (cos, sin) of the cone
// boundaries beta_i = i w, i = 0..n.  The estimate's cone is confirmed, or
// moved, with FP64 side tests, sin(angle - beta) r = Y cos(beta) - X sin(beta),
// so that the index is floor(angle / w) except at rounding distance from a
// boundary (where the relevant-cone marking also holds the neighbour); the
// local coordinate comes from the FP32 angle between the point and the
// cone's lower boundary.
__device__ __forceinline__ int angle_select(double X, double Y, float est, double rw, int n,
                                            bool periodic, const double* bnd, float& u) {
  IFGF_NO_CONTRACT
  const double2* b2 = reinterpret_cast<const double2*>(bnd);
  int i = min((int)(est * (float)rw), n - 1);
  // Boundaries i and i + 1, loaded together (the table has n + 1 entries).
  const double2 b0 = b2[i], b1 = b2[i + 1];
  double cb = b0.x, sb = b0.y;
  double d = Y * cb - X * sb;
  const double d1 = Y * b1.x - X * b1.y;
  if (d < 0.0) {
    // Rare: the estimate is too high (by one cone unless the cones are
    // narrower than its error).
    for (int m = 0; m < n && d < 0.0; ++m) {
      if (i > 0)
        --i;
      else if (periodic)
        i = n - 1;
      else
        break;
      cb = b2[i].x;
      sb = b2[i].y;
      d = Y * cb - X * sb;
    }
  } else if (d1 > 0.0 && i + 1 < n) {
    // Rare: the estimate is too low.
    ++i;
    cb = b1.x;
    sb = b1.y;
    d = d1;
    while (i + 1 < n) {
      const double2 bn = b2[i + 1];
      if (!(Y * bn.x - X * bn.y > 0.0)) break;
      ++i;
      cb = bn.x;
      sb = bn.y;
      d = Y * cb - X * sb;
    }
  }
  const double c = X * cb + Y * sb;
  u = atan2f((float)d, (float)c) * (float)(2.0 * rw) - 1.0f;
  return i;
}

// FP64 mode: cone_coord and cone_index (the rounding path of the relevant-cone
// marking).  FP32-mixed: r, s and the side tests in FP64, the angles'
// estimates and local coordinates in FP32 (the two FP64 arctangents are most
// of the geometry's cost in the per-node propagation).
template <typename T>
__device__ __forceinline__ ConeSel cone_select(const StepDev& S, double h, double y0, double y1,
                                               double y2, T u[3]);
template <>
__device__ __forceinline__ ConeSel cone_select<double>(const StepDev& S, double h, double y0,
                                                       double y1, double y2, double u[3]) {
  const ConeCoord c = cone_coord(S, h, y0, y1, y2);
  const int is = cone_index(c.q[0], S.ns, u[0]);
  const int it = cone_index(c.q[1], S.nt, u[1]);
  const int ip = cone_index(c.q[2], S.np, u[2]);
  return ConeSel{((int64_t)is * S.nt + it) * S.np + ip, c.r, 1.0 / c.r};
}
template <>
__device__ __forceinline__ ConeSel cone_select<float>(const StepDev& S, double h, double y0,
                                                      double y1, double y2, float u[3]) {
  IFGF_NO_CONTRACT
  ConeSel c;
  const double rho2 = y0 * y0 + y1 * y1;
  c.r = sqrt(rho2 + y2 * y2);
  c.rinv = 1.0 / c.r;
  double u0;
  const int is = cone_index(h * c.rinv * S.rds, S.ns, u0);
  u[0] = (float)u0;
  const double rho = sqrt(rho2);
  const float th = atan2_est((float)rho, (float)y2);
  float ph = atan2_est((float)y1, (float)y0);
  if (ph < 0.0f) ph += (float)(2.0 * kPiD);
  const int it = angle_select(y2, rho, th, S.rdt, S.nt, false, S.t_bnd, u[1]);
  const int ip = angle_select(y0, y1, ph, S.rdp, S.np, true, S.p_bnd, u[2]);
  c.gamma = ((int64_t)is * S.nt + it) * S.np + ip;
  return c;
}

// Position of interpolation node (a, b, c) of cone (is, it, ip), relative to
// the centre of its box: (h/s) (sin th cos ph, sin th sin ph, cos th).
template <int PS, int PA>
__device__ __forceinline__ void node_offset(const StepDev& S, double h,
                                            int is, int it, int ip, int a,
                                            int b, int c, double y[3]) {
  IFGF_NO_CONTRACT
  double s = S.s_node[is * PS + a];
  double st = S.t_node[2 * (it * PA + b)];
  double ct = S.t_node[2 * (it * PA + b) + 1];
  double sp = S.p_node[2 * (ip * PA + c)];
  double cp = S.p_node[2 * (ip * PA + c) + 1];
  double r = h / s;
  y[0] = r * st * cp;
  y[1] = r * st * sp;
  y[2] = r * ct;
}

// Lagrange basis at the N first-kind Chebyshev nodes t_m, product form:
// L_j(u) = w_j prod_{m != j} (u - t_m), w_j = 1 / prod_{m != j} (t_j - t_m).
template <int N, typename R>
__device__ __forceinline__ void lagrange(R u, const double* t, const double* w,
                                         R* L) {
  R d[N];
#pragma unroll
  for (int m = 0; m < N; ++m) d[m] = u - (R)t[m];
  R pre[N];
  R acc = (R)1;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    pre[j] = acc;
    acc *= d[j];
  }
  acc = (R)1;
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    L[j] = pre[j] * acc * (R)w[j];
    acc *= d[j];
  }
}

template <typename T> struct C2;
template <> struct C2<double> { typedef double2 type; };
template <> struct C2<float> { typedef float2 type; };

// Tensor contraction sum_{a,b,c} Ls[a] Lt[b] Lp[c] v[(a PA + b) PA + c],
// summed innermost-first (phi, then theta, then s).
template <int PS, int PA, typename T>
__device__ __forceinline__ void contract(const typename C2<T>::type* __restrict__ v,
                                         const T* Ls, const T* Lt, const T* Lp,
                                         T& re, T& im) {
  T sr = 0, si = 0;
#pragma unroll
  for (int a = 0; a < PS; ++a) {
    T tr = 0, ti = 0;
#pragma unroll
    for (int b = 0; b < PA; ++b) {
      T pr = 0, pi = 0;
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        typename C2<T>::type x = v[(a * PA + b) * PA + c];
        pr += Lp[c] * x.x;
        pi += Lp[c] * x.y;
      }
      tr += Lt[b] * pr;
      ti += Lt[b] * pi;
    }
    sr += Ls[a] * tr;
    si += Ls[a] * ti;
  }
  re = sr;
  im = si;
}

// e^{i phase} for phase = kappa * r given in FP64.  FP64 mode: FP64 sincos.
// FP32-mixed: the number of turns kappa r / (2 pi) is reduced to [-1/2, 1/2]
// in FP64, then the hardware sine and cosine of f turns in FP32 (1.3e-7
// absolute error on gfx950, against 5e-8 for sincospif at about fifteen
// times the instructions).
template <typename T>
__device__ __forceinline__ void expi(double phase, T& c, T& s);
template <>
__device__ __forceinline__ void expi<double>(double phase, double& c, double& s) {
  sincos(phase, &s, &c);
}
template <>
__device__ __forceinline__ void expi<float>(double phase, float& c, float& s) {
  double t = phase * kInv2Pi;
  float f = (float)(t - rint(t));
  s = __builtin_amdgcn_sinf(f);
  c = __builtin_amdgcn_cosf(f);
}

// ---------------------------------------------------------------------------
// Apply kernels.
// ---------------------------------------------------------------------------

// Densities, user layout [rhs][N] -> sorted layout [i][rhs].
// Geometry of node p of parent cone index (is, it, ip) of step l + 1 seen
// from the child in octant o (child box centre at +-H_c/2 per axis from the
// parent's): the child cone alpha, the local coordinates u and the ratio
// G(x_p, x_k)/G(x_p, x_j) (phase reduced in FP64).  Box-independent.
template <int PS, int PA, typename T>
__device__ __forceinline__ int node_octant_geometry(const StepDev& S, const StepDev& Q, double hp,
                                                    double hc, double Hc, double kappa, int is,
                                                    int it, int ip, int o, int p, T u[3],
                                                    typename C2<T>::type& rat) {
  const int a = p / (PA * PA), bb = (p / PA) % PA, cc = p % PA;
  double yp[3];
  node_offset<PS, PA>(Q, hp, is, it, ip, a, bb, cc, yp);
  double y0, y1, y2, rj;
  {
    IFGF_NO_CONTRACT
    y0 = yp[0] - (((o >> 2) & 1) ? 0.5 * Hc : -0.5 * Hc);
    y1 = yp[1] - (((o >> 1) & 1) ? 0.5 * Hc : -0.5 * Hc);
    y2 = yp[2] - ((o & 1) ? 0.5 * Hc : -0.5 * Hc);
    rj = sqrt(yp[0] * yp[0] + yp[1] * yp[1] + yp[2] * yp[2]);
  }
  const ConeSel cr = cone_select<T>(S, hc, y0, y1, y2, u);
  T gcv, gsv;
  expi<T>(kappa * (cr.r - rj), gcv, gsv);
  const T amp = (T)(rj * cr.rinv);
  rat.x = gcv * amp;
  rat.y = gsv * amp;
  return (int)cr.gamma;
}

template <typename T>
__global__ void perm_in_kernel(const typename C2<T>::type* __restrict__ in,
                               typename C2<T>::type* __restrict__ out,
                               const int* __restrict__ perm, int64_t n,
                               int nrhs) {
  int64_t t = gtid();
  if (t >= n * nrhs) return;
  int64_t i = t / nrhs;
  int r = (int)(t - i * nrhs);
  out[t] = in[(int64_t)r * n + perm[i]];
}

template <typename T>
__global__ void perm_out_kernel(const typename C2<T>::type* __restrict__ in,
                                typename C2<T>::type* __restrict__ out,
                                const int* __restrict__ perm, int64_t n,
                                int nrhs) {
  int64_t t = gtid();
  if (t >= n * nrhs) return;
  int64_t i = t / nrhs;
  int r = (int)(t - i * nrhs);
  out[(int64_t)r * n + perm[i]] = in[t];
}

template <typename T>
__global__ void zero_kernel(typename C2<T>::type* __restrict__ p, int64_t n) {
  int64_t t = gtid();
  if (t >= n) return;
  typename C2<T>::type z;
  z.x = 0;
  z.y = 0;
  p[t] = z;
}

// Near field: out[i] = sum over the points m of the level-D neighbour boxes
// of box(i), m != i, of a_m e^{i kappa r}/(4 pi r).
template <typename T, int MAXR>
__global__ void __launch_bounds__(256)
near_field_kernel(ApplyArgs A, typename C2<T>::type* __restrict__ out) {
  int64_t i = gtid();
  if (i >= A.n) return;
  const StepDev& S = A.step[0];
  int b = S.pt_box[i];
  double kappa = A.inst_kappa[S.inst[b]];
  double xi = A.x[i], yi = A.y[i], zi = A.z[i];
  T accr[MAXR], acci[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) accr[r] = acci[r] = 0;
  const T inv4pi = (T)(0.25 / kPiD);
  for (int64_t j = A.nbr_begin[b]; j < A.nbr_begin[b + 1]; ++j) {
    int nb = A.nbr[j];
    int m0 = S.first[nb], m1 = m0 + S.count[nb];
    for (int m = m0; m < m1; ++m) {
      if (m == i) continue;
      T dx = (T)(xi - A.x[m]), dy = (T)(yi - A.y[m]), dz = (T)(zi - A.z[m]);
      T r = sqrt(dx * dx + dy * dy + dz * dz);
      T c, s;
      if constexpr (sizeof(T) == 8) {
        sincos(kappa * (double)r, &s, &c);
      } else {
        sincosf((float)kappa * r, &s, &c);
      }
      T g = inv4pi / r;
      c *= g;
      s *= g;
      const typename C2<T>::type* a = ((const typename C2<T>::type*)A.dens_sorted) + (int64_t)m * A.nrhs;
      for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
        typename C2<T>::type av = a[r2];
        accr[r2] += av.x * c - av.y * s;
        acci[r2] += av.x * s + av.y * c;
      }
    }
  }
  for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
    typename C2<T>::type v;
    v.x = accr[r2];
    v.y = acci[r2];
    out[i * A.nrhs + r2] = v;
  }
}

// LevelDEvaluations: one thread per (relevant leaf cone, node p).
// F_k(x_p) = sum_{x' in B_k} a(x') (|x_p - x_k|/|x_p - x'|)
//            exp(i kappa (|x_p - x'| - |x_p - x_k|)).
template <int PS, int PA, typename T, int MAXR>
__global__ void __launch_bounds__(256)
leaf_eval_kernel(ApplyArgs A, typename C2<T>::type* __restrict__ V) {
  constexpr int P = PS * PA * PA;
  const StepDev& S = A.step[0];
  int64_t t = gtid();
  if (t >= S.ncones * P) return;
  int64_t slot = t / P;
  int p = (int)(t - slot * P);
  unsigned long long key = S.cone_key[slot];
  int64_t b = (int64_t)(key / (unsigned long long)S.ngrid);
  int64_t g = (int64_t)(key - (unsigned long long)b * S.ngrid);
  int is = (int)(g / ((int64_t)S.nt * S.np));
  int it = (int)((g / S.np) % S.nt);
  int ip = (int)(g % S.np);
  int a = p / (PA * PA), bb = (p / PA) % PA, cc = p % PA;
  int inst = S.inst[b];
  double h = S.inst_h[inst];
  double kappa = A.inst_kappa[inst];
  double cx = S.center[3 * b], cy = S.center[3 * b + 1], cz = S.center[3 * b + 2];
  double y[3];
  node_offset<PS, PA>(S, h, is, it, ip, a, bb, cc, y);
  T accr[MAXR], acci[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) accr[r] = acci[r] = 0;
  const int m0 = S.first[b], m1 = m0 + S.count[b];
  typedef typename C2<T>::type CT;
  const CT* dens = (const CT*)A.dens_sorted;
  if constexpr (sizeof(T) == 8) {
    IFGF_NO_CONTRACT
    double x0 = cx + y[0], x1 = cy + y[1], x2 = cz + y[2];
    double e0 = x0 - cx, e1 = x1 - cy, e2 = x2 - cz;
    double rk = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    for (int m = m0; m < m1; ++m) {
      double dx = x0 - A.x[m], dy = x1 - A.y[m], dz = x2 - A.z[m];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      double sn, cs;
      sincos(kappa * (r - rk), &sn, &cs);
      double amp = rk / r;
      cs *= amp;
      sn *= amp;
      for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
        const CT w = dens[(int64_t)m * A.nrhs + r2];
        accr[r2] += w.x * cs - w.y * sn;
        acci[r2] += w.x * sn + w.y * cs;
      }
    }
  } else {
    // Box-relative FP32: y node offset, q source offset (plan-time, with
    // |q|^2); the phase |y - q| - |y| = (|q|^2 - 2 y.q) / (|y - q| + |y|) has
    // no cancellation and is at most the box diameter, so its number of
    // turns is reduced in FP32 and e^{i kappa diff} taken from the hardware
    // sine and cosine.  Quotients by the hardware reciprocal and reciprocal
    // square root (1 ulp).
    const float y0 = (float)y[0], y1 = (float)y[1], y2 = (float)y[2];
    const float ry = sqrtf(y0 * y0 + y1 * y1 + y2 * y2);
    const float kturn = (float)(kappa * kInv2Pi);
    for (int m = m0; m < m1; ++m) {
      const float4 q = A.q_leaf[m];
      const float d0 = y0 - q.x, d1 = y1 - q.y, d2 = y2 - q.z;
      const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const float rinv = __builtin_amdgcn_rsqf(r2);  // 1/|y - q|, and |y - q| = r2 / it
      const float diff =
          (q.w - 2.0f * (y0 * q.x + y1 * q.y + y2 * q.z)) * __builtin_amdgcn_rcpf(r2 * rinv + ry);
      const float turns = kturn * diff;
      const float f = turns - rintf(turns);
      float sn = __builtin_amdgcn_sinf(f), cs = __builtin_amdgcn_cosf(f);
      const float amp = ry * rinv;
      cs *= amp;
      sn *= amp;
      for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
        const CT w = dens[(int64_t)m * A.nrhs + r2];
        accr[r2] += w.x * cs - w.y * sn;
        acci[r2] += w.x * sn + w.y * cs;
      }
    }
  }
  for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
    typename C2<T>::type v;
    v.x = (T)accr[r2];
    v.y = (T)acci[r2];
    V[(slot * A.nrhs + r2) * P + p] = v;
  }
}

// Interpolation(d) at step l: blocks of kInterpParts waves over the same 64
// target points (one per lane), wave w summing the cousin boxes w,
// w + kInterpParts, ... of each target's list; the parts are added in LDS.
// The lanes of a wave still walk their (mostly shared) cousin list in step,
// so a gather instruction touches few cones, and the launch has
// kInterpParts times the waves of one wave per 64 targets.
static constexpr int kInterpParts = 4;

template <int PS, int PA, typename T, int MAXR>
__global__ void __launch_bounds__(64 * kInterpParts)
interp_kernel(ApplyArgs A, int l, const typename C2<T>::type* __restrict__ V,
              typename C2<T>::type* __restrict__ out) {
  typedef typename C2<T>::type CT;
  constexpr int P = PS * PA * PA;
  __shared__ CT s_acc[kInterpParts - 1][MAXR][64];
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int64_t i = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 64 + lane;
  const StepDev& S = A.step[l];
  const int b = i < A.n ? S.pt_box[i] : -1;
  T accr[MAXR], acci[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) accr[r] = acci[r] = 0;
  bool miss = false;  // a cone look-up missed (reported once, after the loop)
  if (b >= 0) {
    const int inst = S.inst[b];
    const double h = S.inst_h[inst];
    const double kappa = A.inst_kappa[inst];
    const double xi = A.x[i], yi = A.y[i], zi = A.z[i];
    for (int64_t j = S.cous_begin[b] + part; j < S.cous_begin[b + 1]; j += kInterpParts) {
      const int k = S.cous[j];
      double y0, y1, y2;
      {
        IFGF_NO_CONTRACT
        y0 = xi - S.center[3 * k];
        y1 = yi - S.center[3 * k + 1];
        y2 = zi - S.center[3 * k + 2];
      }
      // FP64 selection in both modes: the FP32 one's boundary-table loads
      // would sit between the geometry and the look-up in this latency-bound
      // loop.
      double u[3];
      const ConeSel cc = cone_select<double>(S, h, y0, y1, y2, u);
      const unsigned long long key =
          (unsigned long long)k * S.ngrid + (unsigned long long)cc.gamma;
      const int slot = cone_lookup(S, key);
      if (slot < 0) {
        miss = true;
        continue;
      }
      T Ls[PS], Lt[PA], Lp[PA];
      lagrange<PS, T>((T)u[0], A.cheb.ts, A.cheb.ws, Ls);
      lagrange<PA, T>((T)u[1], A.cheb.ta, A.cheb.wa, Lt);
      lagrange<PA, T>((T)u[2], A.cheb.ta, A.cheb.wa, Lp);
      T gc, gs;
      expi<T>(kappa * cc.r, gc, gs);
      const T amp = (T)((0.25 / kPiD) * cc.rinv);
      gc *= amp;
      gs *= amp;
      const CT* vb = V + (int64_t)slot * A.nrhs * P;
      for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
        T vr, vi;
        contract<PS, PA, T>(vb + r2 * P, Ls, Lt, Lp, vr, vi);
        accr[r2] += vr * gc - vi * gs;
        acci[r2] += vr * gs + vi * gc;
      }
    }
  }
  if (miss) atomicOr(A.err, 1);
  if (part > 0) {
#pragma unroll
    for (int r = 0; r < MAXR; ++r) s_acc[part - 1][r][lane] = CT{accr[r], acci[r]};
  }
  __syncthreads();
  if (part > 0 || b < 0) return;
#pragma unroll
  for (int q = 0; q < kInterpParts - 1; ++q)
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      accr[r] += s_acc[q][r][lane].x;
      acci[r] += s_acc[q][r][lane].y;
    }
  for (int r2 = 0; r2 < A.nrhs && r2 < MAXR; ++r2) {
    CT v = out[i * A.nrhs + r2];
    v.x += accr[r2];
    v.y += acci[r2];
    out[i * A.nrhs + r2] = v;
  }
}

// Propagation from step l to step l + 1, one thread per (relevant parent
// cone, node p), one wave per block, with the child cone values staged in
// LDS: per child octant the lanes' child cones are collected (wave ballots;
// the nodes of a parent cone fall into few child cones), up to kNodeBufs of
// them are copied into LDS with contiguous loads, kNodeStageBatch cones'
// loads in flight together (one memory latency per batch instead of per
// cone), and each lane contracts its cone's values from there (from global
// memory beyond kNodeBufs).
static constexpr int kNodeBufs = 8;
static constexpr int kNodeStageBatch = 2;

template <int PS, int PA, typename T, int MAXR>
__global__ void __launch_bounds__(64)
prop_node_kernel(ApplyArgs A, int l, const typename C2<T>::type* __restrict__ Vc,
                 typename C2<T>::type* __restrict__ Vp) {
  typedef typename C2<T>::type CT;
  constexpr int P = PS * PA * PA;
  __shared__ CT s_v[kNodeBufs][MAXR * P];
  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  const int64_t n = Q.ncones * P;
  const int64_t t0 = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * 64;
  if (t0 >= n) return;  // the whole wave is past the end
  const int lane = threadIdx.x;
  const int64_t t = t0 + lane;
  const bool active = t < n;
  const int nrhs = A.nrhs;
  const int64_t slot = active ? t / P : 0;
  const int p = active ? (int)(t - slot * P) : 0;
  const unsigned long long key = Q.cone_key[slot];
  const int64_t j = (int64_t)(key / (unsigned long long)Q.ngrid);
  const int64_t g = (int64_t)(key - (unsigned long long)j * Q.ngrid);
  const int is = (int)(g / ((int64_t)Q.nt * Q.np));
  const int it = (int)((g / Q.np) % Q.nt);
  const int ip = (int)(g % Q.np);
  const int a = p / (PA * PA), bb = (p / PA) % PA, cc = p % PA;
  const int inst = Q.inst[j];
  const double hp = Q.inst_h[inst];
  const double hc = S.inst_h[inst];
  const double kappa = A.inst_kappa[inst];
  const double cjx = Q.center[3 * j], cjy = Q.center[3 * j + 1], cjz = Q.center[3 * j + 2];
  double yp[3];
  node_offset<PS, PA>(Q, hp, is, it, ip, a, bb, cc, yp);
  double x0, x1, x2, rj;
  {
    IFGF_NO_CONTRACT
    x0 = cjx + yp[0];
    x1 = cjy + yp[1];
    x2 = cjz + yp[2];
    double e0 = x0 - cjx, e1 = x1 - cjy, e2 = x2 - cjz;
    rj = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  }
  T accr[MAXR], acci[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) accr[r] = acci[r] = 0;
  bool miss = false;  // a cone look-up missed (reported once, after the loop)
  for (int o = 0; o < 8; ++o) {
    const int k = active ? Q.child[8 * j + o] : -1;
    int cslot = -1;
    T Ls[PS], Lt[PA], Lp[PA];
    T gc = 0, gs = 0;
    if (k >= 0) {
      double y0, y1, y2;
      {
        IFGF_NO_CONTRACT
        y0 = x0 - S.center[3 * k];
        y1 = x1 - S.center[3 * k + 1];
        y2 = x2 - S.center[3 * k + 2];
      }
      T u[3];
      const ConeSel c = cone_select<T>(S, hc, y0, y1, y2, u);
      const unsigned long long ckey =
          (unsigned long long)k * S.ngrid + (unsigned long long)c.gamma;
      cslot = cone_lookup(S, ckey);
      miss |= cslot < 0;
      lagrange<PS, T>(u[0], A.cheb.ts, A.cheb.ws, Ls);
      lagrange<PA, T>(u[1], A.cheb.ta, A.cheb.wa, Lt);
      lagrange<PA, T>(u[2], A.cheb.ta, A.cheb.wa, Lp);
      // G(x, x_k) / G(x, x_j) = (r_j / r_k) e^{i kappa (r_k - r_j)}.
      expi<T>(kappa * (c.r - rj), gc, gs);
      const T amp = (T)(rj * c.rinv);
      gc *= amp;
      gs *= amp;
    }
    // Stage the distinct child cones of the wave in LDS: collect them with
    // ballots (lane q keeps the slot of the q-th), then copy them
    // kNodeStageBatch cones at a time with all their loads in flight
    // (clamped indices: every load is in bounds; stores past the end are
    // skipped).
    unsigned long long pend = __ballot(cslot >= 0);
    if (pend == 0ull) continue;
    int buf = -1, nb = 0, qslot = -1;
    while (pend) {
      const int c = __shfl(cslot, __ffsll((long long)pend) - 1);
      const bool mine = cslot == c;
      if (nb < kNodeBufs) {
        if (lane == nb) qslot = c;
        if (mine) buf = nb;
        ++nb;
      }
      pend &= ~__ballot(mine);
    }
    {
      constexpr int NCH = (MAXR * P + 63) / 64;  // lane-strided chunks per cone
      constexpr int QB = MAXR == 1 ? kNodeStageBatch : 1;
      const int len = nrhs * P;
      for (int q0 = 0; q0 < nb; q0 += QB) {
        CT tmp[QB][NCH];
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) {
          const CT* src = Vc + (int64_t)__shfl(qslot, min(q0 + qq, nb - 1)) * len;
#pragma unroll
          for (int h = 0; h < NCH; ++h) tmp[qq][h] = src[min(h * 64 + lane, len - 1)];
        }
#pragma unroll
        for (int qq = 0; qq < QB; ++qq)
#pragma unroll
          for (int h = 0; h < NCH; ++h)
            if (q0 + qq < nb && h * 64 + lane < len) s_v[q0 + qq][h * 64 + lane] = tmp[qq][h];
      }
    }
    __syncthreads();  // one wave: the LDS copies are complete
    if (cslot >= 0) {
      const CT* vb = buf >= 0 ? nullptr : Vc + (int64_t)cslot * nrhs * P;
      for (int r2 = 0; r2 < nrhs && r2 < MAXR; ++r2) {
        T vr, vi;
        if (buf >= 0)
          contract<PS, PA, T>(&s_v[buf][r2 * P], Ls, Lt, Lp, vr, vi);
        else
          contract<PS, PA, T>(vb + r2 * P, Ls, Lt, Lp, vr, vi);
        accr[r2] += vr * gc - vi * gs;
        acci[r2] += vr * gs + vi * gc;
      }
    }
    __syncthreads();  // the buffers are reused by the next octant
  }
  if (miss) atomicOr(A.err, 1);
  if (!active) return;
  for (int r2 = 0; r2 < nrhs && r2 < MAXR; ++r2) {
    CT v;
    v.x = accr[r2];
    v.y = acci[r2];
    Vp[(slot * nrhs + r2) * P + p] = v;
  }
}

// Matrix-core (MFMA 16x16x4) operand layouts on gfx950, one wave:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[row(l, r)][l % 16], r = 0..3, with
//                row = 4 (l / 16) + r for FP32 and 4 r + l / 16 for FP64.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};

// Boxes per chunk of the grouped propagation (columns of the GEMM are
// (box, right-hand side) pairs; 32 FP32 or 16 FP64 columns per chunk).
static constexpr int kMfmaThreads = 256;

template <typename T, int MAXR>
struct ChunkCols {
  static constexpr int boxes = (sizeof(T) == 4 ? 32 : 16) / MAXR;
};

// Propagation as batched small GEMMs on the matrix cores.  One block (4
// waves) per chunk of parent cones sharing (instance, gamma'), processed
// in sub-chunks of CB boxes.  The node geometry -- the child cone alpha,
// the local coordinates u and the ratio G(x,x_k)/G(x,x_j) of node p of
// gamma' seen from the child in octant o -- does not depend on the box and
// is computed once per block.  For every octant o and child cone alpha,
// the nodes p with alpha(p) = alpha are the rows of
//     C[p][(box, rhs)] = sum_q W[p][q] X[q][(box, rhs)],
//     W[p][q] = L_a(u_s(p)) L_b(u_theta(p)) L_c(u_phi(p)),  q = (a, b, c),
// X holding the child cone values of the boxes' children in octant o; the
// product runs on 16x16x4 MFMA tiles and ratio(p) * C accumulates per
// (box, p) in LDS.  The block owns its parent cones: no atomics.
template <int PS, int PA, typename T, int MAXR>
__global__ void __launch_bounds__(kMfmaThreads)
prop_mfma_kernel(ApplyArgs A, int l, const typename C2<T>::type* __restrict__ Vc,
                 typename C2<T>::type* __restrict__ Vp) {
  typedef typename C2<T>::type CT;
  typedef typename Mfma<T>::v4 V4;
  constexpr int P = PS * PA * PA;
  static_assert(P <= 128, "two nodes per lane");
  constexpr int NW = PS + 2 * PA;
  constexpr int KP = (P + 3) / 4 * 4;
  constexpr int CB = ChunkCols<T, MAXR>::boxes;
  constexpr int NCOL = CB * MAXR;  // <= 32 columns
  constexpr int NAMAX = 8;         // child cones per octant with a cached slot
  constexpr int KS = (KP / 4 + 3) / 4 * 4;  // k-steps, padded to whole 4-vectors
  constexpr int RS = 4 * KS + 4;            // row stride of s_A (bank offset)
  typedef T T4 __attribute__((ext_vector_type(4)));
  __shared__ T s_u[8 * P * 3];            // local coordinates of (o, p)
  __shared__ T s_L[P * NW];               // Lagrange weights of one octant
  // Interpolation matrix of one octant: row pos (the node at position pos
  // of the octant's grouping by child cone), entry q at [q % 4][q / 4],
  // zero for q >= P.
  __shared__ __attribute__((aligned(16))) T s_A[P * RS];
  __shared__ T s_rat[8 * P * 2];
  __shared__ int s_dist[8 * P];           // distinct child cones per octant
  __shared__ unsigned char s_rows[8 * P]; // nodes of octant o grouped by alpha
  __shared__ int s_rbeg[8 * (P + 1)];
  __shared__ int s_na[8];
  // The output accumulators; during set-up the same memory holds the child
  // cone alpha of every (o, p).
  static_assert(NCOL * P * 2 * sizeof(T) >= 8 * P * sizeof(int), "alias");
  __shared__ T s_y[NCOL * P * 2];
  int* const s_alpha = reinterpret_cast<int*>(s_y);
  __shared__ int s_pslot[CB], s_box[CB];
  __shared__ int s_nlist[8 * CB], s_child[8 * CB], s_no[8], s_ipre[9];
  __shared__ int s_cslot[8 * CB * NAMAX];

  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  constexpr int NWAVES = kMfmaThreads / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nrhs = A.nrhs;
  const int64_t c = blockIdx.x;
  const int64_t g0 = Q.chunk_start[c];
  const int nchunk = Q.chunk_len[c];
  const unsigned long long key0 = Q.cone_key[Q.gslot[g0]];
  const int64_t j0 = (int64_t)(key0 / (unsigned long long)Q.ngrid);
  const int64_t g = (int64_t)(key0 - (unsigned long long)j0 * Q.ngrid);
  const int is = (int)(g / ((int64_t)Q.nt * Q.np));
  const int it = (int)((g / Q.np) % Q.nt);
  const int ip = (int)(g % Q.np);
  const int inst = Q.inst[j0];
  const double hp = Q.inst_h[inst];
  const double hc = S.inst_h[inst];
  const double Hc = S.inst_H[inst];
  const double kappa = A.inst_kappa[inst];

  // The zero padding of s_A (columns q >= P), written once.
  for (int i = tid; i < P * (4 * KS - P); i += blockDim.x) {
    const int pos = i / (4 * KS - P), q = P + i % (4 * KS - P);
    s_A[pos * RS + (q & 3) * KS + (q >> 2)] = 0;
  }
  // Node geometry, once per block.
  for (int i = tid; i < 8 * P; i += blockDim.x) {
    const int o = i / P, p = i - (i / P) * P;
    T u[3];
    typename C2<T>::type rat;
    s_alpha[i] = node_octant_geometry<PS, PA, T>(S, Q, hp, hc, Hc, kappa, is, it, ip, o, p, u, rat);
    s_u[3 * i] = u[0];
    s_u[3 * i + 1] = u[1];
    s_u[3 * i + 2] = u[2];
    s_rat[2 * i] = rat.x;
    s_rat[2 * i + 1] = rat.y;
  }
  __syncthreads();
  // Per octant (wave w: octants w and w + 4), the distinct child cones and
  // the nodes grouped by child cone, with wave ballots; lane holds nodes
  // lane and lane + 64.
  for (int o = wave; o < 8; o += NWAVES) {
    const bool has0 = lane < P, has1 = lane + 64 < P;
    const int a0 = has0 ? s_alpha[o * P + lane] : -1;
    const int a1 = has1 ? s_alpha[o * P + lane + 64] : -1;
    bool f0 = has0, f1 = has1;
    int k0 = 0, k1 = 0, na = 0;
    for (;;) {
      const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
      if (m0 == 0ull && m1 == 0ull) break;
      const int lead = m0 ? __shfl(a0, __ffsll((long long)m0) - 1)
                          : __shfl(a1, __ffsll((long long)m1) - 1);
      if (f0 && a0 == lead) { k0 = na; f0 = false; }
      if (f1 && a1 == lead) { k1 = na; f1 = false; }
      if (lane == 0) s_dist[o * P + na] = lead;
      ++na;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
    int base = 0;
    for (int k = 0; k < na; ++k) {
      const unsigned long long m0 = __ballot(has0 && k0 == k), m1 = __ballot(has1 && k1 == k);
      if (has0 && k0 == k) s_rows[o * P + base + __popcll(m0 & lt)] = (unsigned char)lane;
      if (has1 && k1 == k)
        s_rows[o * P + base + __popcll(m0) + __popcll(m1 & lt)] = (unsigned char)(lane + 64);
      if (lane == 0) s_rbeg[o * (P + 1) + k] = base;
      base += __popcll(m0) + __popcll(m1);
    }
    if (lane == 0) {
      s_rbeg[o * (P + 1) + na] = base;
      s_na[o] = na;
    }
  }
  __syncthreads();

  const int kq = lane >> 4;
  for (int sub = 0; sub * CB < nchunk; ++sub) {
    const int nbk = min(CB, nchunk - sub * CB);
    if (tid < nbk) {
      const int ps = Q.gslot[g0 + sub * CB + tid];
      s_pslot[tid] = ps;
      s_box[tid] = (int)(Q.cone_key[ps] / (unsigned long long)Q.ngrid);
    }
    for (int i = tid; i < NCOL * P * 2; i += blockDim.x) s_y[i] = 0;
    __syncthreads();
    // Children present per octant, compacted with a wave ballot.
    for (int o = wave; o < 8; o += NWAVES) {
      const int k = lane < nbk ? Q.child[8 * (int64_t)s_box[lane] + o] : -1;
      const unsigned long long mask = __ballot(k >= 0);
      if (k >= 0) {
        const int pos = __popcll(mask & ((1ull << lane) - 1ull));
        s_nlist[o * CB + pos] = lane;
        s_child[o * CB + pos] = k;
      }
      if (lane == 0) s_no[o] = __popcll(mask);
    }
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int o = 0; o < 8; ++o) {
        s_ipre[o] = acc;
        acc += s_na[o] * ((s_no[o] * nrhs + 15) / 16);
      }
      s_ipre[8] = acc;
    }
    // Child cone slots of every (octant, box, child cone), in one batch.
    for (int idx = tid; idx < 8 * CB * NAMAX; idx += blockDim.x) {
      const int o = idx / (CB * NAMAX), rem = idx - o * (CB * NAMAX);
      const int n = rem / NAMAX, k = rem - n * NAMAX;
      int cs = -1;
      if (n < s_no[o] && k < s_na[o]) {
        cs = cone_lookup(S, (unsigned long long)s_child[o * CB + n] * S.ngrid + s_dist[o * P + k]);
        if (cs < 0) atomicOr(A.err, 1);
      }
      s_cslot[idx] = cs;
    }
    __syncthreads();
    // Octant by octant (all waves on one octant, so every (box, node) of
    // the output is updated by one lane at a time: plain LDS
    // read-modify-write).  Operands need no masks: a padded column reads a
    // valid cone and is never stored, a padded row reads a valid row of
    // s_A and is never stored, and the padded K entries of s_A are 0.
    for (int o = 0; o < 8; ++o) {
      const int no = s_no[o];
      if (no == 0) continue;  // uniform across the block
      const int ncols = no * nrhs;
      const int ntn = (ncols + 15) / 16;
      const int na = s_na[o];
      // Lagrange weights of this octant's nodes, in grouped order.
      for (int pos = tid; pos < P; pos += blockDim.x) {
        const int p = s_rows[o * P + pos];
        const T* u = s_u + 3 * (o * P + p);
        T* L = s_L + pos * NW;
        lagrange<PS, T>(u[0], A.cheb.ts, A.cheb.ws, L);
        lagrange<PA, T>(u[1], A.cheb.ta, A.cheb.wa, L + PS);
        lagrange<PA, T>(u[2], A.cheb.ta, A.cheb.wa, L + PS + PA);
      }
      __syncthreads();
      // W[p][q] = L_a L_b L_c for q = (a, b, c): one (pos, a, b) per thread.
      for (int i = tid; i < P * PS * PA; i += blockDim.x) {
        const int pos = i / (PS * PA), ab = i - (i / (PS * PA)) * (PS * PA);
        const int a = ab / PA, bq = ab - (ab / PA) * PA;
        const T* L = s_L + pos * NW;
        const T lab = L[a] * L[PS + bq];
        T* Ar = s_A + pos * RS;
#pragma unroll
        for (int cq = 0; cq < PA; ++cq) {
          const int q = (a * PA + bq) * PA + cq;
          Ar[(q & 3) * KS + (q >> 2)] = lab * L[PS + PA + cq];
        }
      }
      __syncthreads();
      // M-tiles of all child cones of this octant, enumerated in order.
      int nmt = 0;
      for (int k = 0; k < na; ++k)
        nmt += (s_rbeg[o * (P + 1) + k + 1] - s_rbeg[o * (P + 1) + k] + 15) / 16;
      // Work items (child cone k, M-tile, N-tile).
      for (int item = wave; item < nmt * ntn; item += NWAVES) {
        const int gm = item / ntn, nt = item - (item / ntn) * ntn;
        int k = 0, mt0 = gm;
        for (;;) {
          const int t = (s_rbeg[o * (P + 1) + k + 1] - s_rbeg[o * (P + 1) + k] + 15) / 16;
          if (mt0 < t) break;
          mt0 -= t;
          ++k;
        }
        const int rb0 = s_rbeg[o * (P + 1) + k], rlen = s_rbeg[o * (P + 1) + k + 1] - rb0;
        const int col = nt * 16 + (lane & 15);
        const bool colok = col < ncols;
        const int n = colok ? col / nrhs : 0;
        const int r = colok ? col - n * nrhs : 0;
        int cs;
        if (k < NAMAX) {
          cs = s_cslot[(o * CB + n) * NAMAX + k];
        } else {
          cs = cone_lookup(
              S, (unsigned long long)s_child[o * CB + n] * S.ngrid + s_dist[o * P + k]);
          if (cs < 0) atomicOr(A.err, 1);
        }
        // B operand: lane holds X[4 kk + kq][col].
        const CT* vp = Vc + ((int64_t)(cs >= 0 ? cs : 0) * nrhs + r) * P + kq;
        T br[KP / 4], bi[KP / 4];
#pragma unroll
        for (int kk = 0; kk < KP / 4; ++kk) {
          const CT x = (4 * kk + 3 < P) ? vp[4 * kk] : vp[min(4 * kk, P - 1 - kq)];
          br[kk] = x.x;
          bi[kk] = x.y;
        }
        const int b = s_nlist[o * CB + n];
        {
          const int mt = mt0;
          // A operand: lane holds W[row 16 mt + lane % 16][4 kk + kq].
          const int arow = min(rb0 + mt * 16 + (lane & 15), P - 1);
          const T4* ap = reinterpret_cast<const T4*>(s_A + arow * RS + kq * KS);
          T av[KS];
#pragma unroll
          for (int j = 0; j < KS / 4; ++j) {
            const T4 v = ap[j];
            av[4 * j] = v.x;
            av[4 * j + 1] = v.y;
            av[4 * j + 2] = v.z;
            av[4 * j + 3] = v.w;
          }
          // Epilogue operands, fetched before the products.
          int pe[4];
          T gce[4], gse[4];
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int mm = mt * 16 + Mfma<T>::row(lane, r4);
            pe[r4] = mm < rlen ? (int)s_rows[o * P + rb0 + mm] : -1;
            const int pp = pe[r4] >= 0 ? pe[r4] : 0;
            gce[r4] = s_rat[2 * (o * P + pp)];
            gse[r4] = s_rat[2 * (o * P + pp) + 1];
          }
          V4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < KP / 4; ++kk) {
            accr = Mfma<T>::mma(av[kk], br[kk], accr);
            acci = Mfma<T>::mma(av[kk], bi[kk], acci);
          }
          // Rows -> nodes, columns -> (box, rhs); times the ratio.
          if (colok) {
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4) {
              if (pe[r4] >= 0) {
                T* y = s_y + 2 * ((b * MAXR + r) * P + pe[r4]);
                y[0] += accr[r4] * gce[r4] - acci[r4] * gse[r4];
                y[1] += accr[r4] * gse[r4] + acci[r4] * gce[r4];
              }
            }
          }
        }
      }
      __syncthreads();
    }
    __syncthreads();
    // Write the parent cones of this sub-chunk.
    for (int idx = tid; idx < nbk * nrhs * P; idx += blockDim.x) {
      const int b = idx / (nrhs * P);
      const int rem = idx - b * (nrhs * P);
      const int r = rem / P, p = rem - (rem / P) * P;
      CT v;
      v.x = s_y[2 * ((b * MAXR + r) * P + p)];
      v.y = s_y[2 * ((b * MAXR + r) * P + p) + 1];
      Vp[((int64_t)s_pslot[b] * nrhs + r) * P + p] = v;
    }
    __syncthreads();
  }
}

// FP32 propagation on the matrix cores, large blocks.  A block of 8 waves
// takes one chunk of parent cones sharing (instance, gamma') and works
// through it in sub-chunks of CB boxes.  The node geometry and the Lagrange
// weights of all eight octants are computed once per block.  Per sub-chunk,
// octant by octant: the interpolation matrix W of the octant is formed in
// LDS (rows in the octant's grouping of nodes by child cone), then every
// wave runs work items (child cone k, M-tile, N-tile) of
//     C[p][(box, rhs)] = sum_q W[p][q] X[q][(box, rhs)]
// on 16x16x4 MFMA tiles, the columns being all boxes of the sub-chunk with
// a child in the octant, and accumulates ratio(p) * C in LDS.  Each wave
// keeps the B tile of its next item in flight while it computes the
// current one; the child cone slots of the next octant are looked up
// during the current octant's items.
template <int PS, int PA, int MAXR>
struct BigProp {
  static constexpr int P = PS * PA * PA;
  static constexpr int NW = PS + 2 * PA;
  static constexpr int NK = (P + 3) / 4;          // k-steps of 4
  static constexpr int KS = (NK + 3) / 4 * 4;     // k-steps padded to whole 4-vectors
  static constexpr int RS = 4 * KS + 4;           // row stride of the W matrix (bank offset)
  static constexpr int NWV = 8;
  static constexpr int CB = 128 / MAXR;           // boxes per sub-chunk
  static constexpr int NCOL = CB * MAXR;          // <= 128 columns
  static constexpr int NAMAX = 8;                 // child cones per octant with a cached slot
  // K order: k-steps 2m and 2m + 1 give lane group kq the adjacent nodes
  // q = 8m + 2kq and 8m + 2kq + 1 (one 16-byte load of two complex
  // values); an odd last k-step gives it q = 8 NPAIR + kq.
  static constexpr int NPAIR = NK / 2;
  static __device__ __forceinline__ int kstep(int q) {
    return q < 8 * NPAIR ? 2 * (q >> 3) + (q & 1) : NK - 1;
  }
  static __device__ __forceinline__ int kgroup(int q) {
    return q < 8 * NPAIR ? (q & 7) >> 1 : q - 8 * NPAIR;
  }
};

// Decodes work item `item` of octant o (M-tiles of all child cones in
// order, times N-tiles) into child cone k, row range and tile indices.
// Decodes work item `item` of octant o (pairs of M-tiles of every child
// cone in order, times N-tiles) into child cone k, first M-tile mt (even)
// and N-tile nt.
template <int P>
__device__ __forceinline__ void big_item(const int* rbeg, int item, int ntn, int& k, int& mt,
                                         int& nt) {
  const int gm = item / ntn;
  nt = item - gm * ntn;
  k = 0;
  int mp = gm;
  for (;;) {
    const int t = (rbeg[k + 1] - rbeg[k] + 31) / 32;
    if (mp < t) break;
    mp -= t;
    ++k;
  }
  mt = 2 * mp;
}

template <int PS, int PA, int MAXR>
__device__ __forceinline__ void big_load_b(const StepDev& S, const float2* __restrict__ Vc,
                                           int* err, const int* cs_tab, const int* ch_tab,
                                           const int* dist, const int* rbeg, int item, int ntn,
                                           int ncols, int nrhs, int lane, bool live, float* br,
                                           float* bi) {
  typedef BigProp<PS, PA, MAXR> B;
  constexpr int P = B::P;
  int k, mt, nt;
  big_item<P>(rbeg, item, ntn, k, mt, nt);
  const int col = nt * 16 + (lane & 15), kq = lane >> 4;
  const int n0 = col / nrhs;
  const int n = col < ncols ? n0 : 0;
  const int r = col < ncols ? col - n0 * nrhs : 0;
  int cs;
  if (k < B::NAMAX) {
    cs = cs_tab[n * B::NAMAX + k];
  } else {
    cs = cone_lookup(S, (unsigned long long)ch_tab[n] * S.ngrid + dist[k]);
    if (cs < 0) atomicOr(err, 1);
  }
  const float2* vp = live ? Vc + ((int64_t)(cs >= 0 ? cs : 0) * nrhs + r) * P : Vc;
  typedef float v4u __attribute__((ext_vector_type(4), aligned(8)));
#pragma unroll
  for (int m = 0; m < B::NPAIR; ++m) {
    if (8 * m + 7 < P) {
      const v4u x = *reinterpret_cast<const v4u*>(vp + 8 * m + 2 * kq);
      br[2 * m] = x.x;
      bi[2 * m] = x.y;
      br[2 * m + 1] = x.z;
      bi[2 * m + 1] = x.w;
    } else {
      const float2 x0 = vp[min(8 * m + 2 * kq, P - 1)];
      const float2 x1 = vp[min(8 * m + 2 * kq + 1, P - 1)];
      br[2 * m] = x0.x;
      bi[2 * m] = x0.y;
      br[2 * m + 1] = x1.x;
      bi[2 * m + 1] = x1.y;
    }
  }
  if constexpr (B::NK & 1) {
    const float2 x = vp[min(8 * B::NPAIR + kq, P - 1)];
    br[B::NK - 1] = x.x;
    bi[B::NK - 1] = x.y;
  }
}

// Accumulates ratio(p) * C of one 16 x 16 tile (rows of lane: pe, ratio
// gc + i gs) into the LDS accumulators; the four reads go before the four
// writes (distinct addresses).
template <typename V4>
__device__ __forceinline__ void big_epilogue(float* s_y, int yb, bool colok, const int* pe,
                                             const float* gc, const float* gs, const V4& accr,
                                             const V4& acci) {
  if (!colok) return;
  float y0[4], y1[4];
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    y0[r4] = 0.f;
    y1[r4] = 0.f;
    if (pe[r4] >= 0) {
      y0[r4] = s_y[2 * (yb + pe[r4])];
      y1[r4] = s_y[2 * (yb + pe[r4]) + 1];
    }
  }
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    if (pe[r4] >= 0) {
      s_y[2 * (yb + pe[r4])] = y0[r4] + accr[r4] * gc[r4] - acci[r4] * gs[r4];
      s_y[2 * (yb + pe[r4]) + 1] = y1[r4] + accr[r4] * gs[r4] + acci[r4] * gc[r4];
    }
  }
}

// One work item: M-tiles mt and (if it exists) mt + 1 of child cone k,
// N-tile nt, sharing the B tile.
template <int PS, int PA, int MAXR>
__device__ __forceinline__ void big_compute(const float* s_A, const float* rat,
                                            const unsigned char* rows, const int* rbeg,
                                            const unsigned char* nl, float* s_y, int item, int ntn,
                                            int ncols, int nrhs, int lane, const float* br,
                                            const float* bi) {
  typedef BigProp<PS, PA, MAXR> B;
  constexpr int P = B::P;
  typedef float v4 __attribute__((ext_vector_type(4)));
  int k, mt, nt;
  big_item<P>(rbeg, item, ntn, k, mt, nt);
  const int rb0 = rbeg[k], rlen = rbeg[k + 1] - rb0;
  const int col = nt * 16 + (lane & 15), kq = lane >> 4;
  const bool colok = col < ncols;
  const int n0 = col / nrhs;
  const int r = col - n0 * nrhs;
  const int yb = colok ? ((int)nl[n0] * MAXR + r) * P : 0;
  const bool two = (mt + 1) * 16 < rlen;  // uniform across the wave
  // A operands: lane holds W[row 16 t + lane % 16][q] with q the node of
  // k-step kk for lane group kq, t = mt, mt + 1.
  float av0[B::KS], av1[B::KS];
  {
    const int arow0 = min(rb0 + mt * 16 + (lane & 15), P - 1);
    const int arow1 = min(rb0 + mt * 16 + 16 + (lane & 15), P - 1);
    const v4* ap0 = reinterpret_cast<const v4*>(s_A + arow0 * B::RS + kq * B::KS);
    const v4* ap1 = reinterpret_cast<const v4*>(s_A + arow1 * B::RS + kq * B::KS);
#pragma unroll
    for (int j = 0; j < B::KS / 4; ++j) {
      const v4 v = ap0[j];
      av0[4 * j] = v.x;
      av0[4 * j + 1] = v.y;
      av0[4 * j + 2] = v.z;
      av0[4 * j + 3] = v.w;
    }
    if (two) {
#pragma unroll
      for (int j = 0; j < B::KS / 4; ++j) {
        const v4 v = ap1[j];
        av1[4 * j] = v.x;
        av1[4 * j + 1] = v.y;
        av1[4 * j + 2] = v.z;
        av1[4 * j + 3] = v.w;
      }
    }
  }
  int pe0[4], pe1[4];
  float gc0[4], gs0[4], gc1[4], gs1[4];
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const int mm0 = mt * 16 + 4 * (lane >> 4) + r4;
    const int mm1 = mm0 + 16;
    const int pos0 = rb0 + (mm0 < rlen ? mm0 : 0);
    const int pos1 = rb0 + (mm1 < rlen ? mm1 : 0);
    pe0[r4] = mm0 < rlen ? (int)rows[pos0] : -1;
    pe1[r4] = mm1 < rlen ? (int)rows[pos1] : -1;
    gc0[r4] = rat[2 * pos0];
    gs0[r4] = rat[2 * pos0 + 1];
    gc1[r4] = rat[2 * pos1];
    gs1[r4] = rat[2 * pos1 + 1];
  }
  if (two) {
    v4 ar0 = {0, 0, 0, 0}, ai0 = {0, 0, 0, 0}, ar1 = {0, 0, 0, 0}, ai1 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < B::NK; ++kk) {
      ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], br[kk], ar0, 0, 0, 0);
      ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], bi[kk], ai0, 0, 0, 0);
      ar1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[kk], br[kk], ar1, 0, 0, 0);
      ai1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[kk], bi[kk], ai1, 0, 0, 0);
    }
    big_epilogue(s_y, yb, colok, pe0, gc0, gs0, ar0, ai0);
    big_epilogue(s_y, yb, colok, pe1, gc1, gs1, ar1, ai1);
  } else {
    v4 ar0 = {0, 0, 0, 0}, ai0 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < B::NK; ++kk) {
      ar0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], br[kk], ar0, 0, 0, 0);
      ai0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], bi[kk], ai0, 0, 0, 0);
    }
    big_epilogue(s_y, yb, colok, pe0, gc0, gs0, ar0, ai0);
  }
}

template <int PS, int PA, int MAXR>
__global__ void __launch_bounds__(512)
prop_big_kernel(ApplyArgs A, int l, const float2* __restrict__ Vc, float2* __restrict__ Vp) {
  typedef BigProp<PS, PA, MAXR> B;
  constexpr int P = B::P, NW = B::NW, KS = B::KS, RS = B::RS, CB = B::CB, NAMAX = B::NAMAX;
  constexpr int NWV = B::NWV;
  static_assert(P <= 128, "two nodes per lane");
  __shared__ float s_L[8 * P * NW];                  // weights of (o, pos)
  __shared__ __attribute__((aligned(16))) float s_A[P * RS];
  __shared__ float s_rat[8 * P * 2];                 // ratio of (o, pos)
  __shared__ unsigned char s_rows[8 * P];            // node p at (o, pos)
  __shared__ int s_rbeg[8 * (P + 1)];
  __shared__ int s_dist[8 * P];
  __shared__ int s_na[8];
  // Accumulators of a sub-chunk; during the set-up the same memory holds
  // the child cone alpha, local coordinates u and ratio of every (o, p).
  __shared__ float s_y[B::NCOL * P * 2];
  static_assert(B::NCOL * P * 2 >= 8 * P * 6, "set-up scratch");
  int* const s_alpha = reinterpret_cast<int*>(s_y);
  float* const s_u = s_y + 8 * P;
  float* const s_ratp = s_y + 8 * P * 4;
  __shared__ int s_pslot[CB], s_box[CB];
  __shared__ int s_child[8][CB];                     // children per octant, compacted
  __shared__ unsigned char s_nl[8][CB];              // their box index in the sub-chunk
  __shared__ int s_no[8];
  __shared__ int s_cs[2][CB * NAMAX];                // child cone slots, two octants

  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nrhs = A.nrhs;
  const int64_t c = blockIdx.x;
  const int64_t g0 = Q.chunk_start[c];
  const int nchunk = Q.chunk_len[c];
  const unsigned long long key0 = Q.cone_key[Q.gslot[g0]];
  const int64_t j0 = (int64_t)(key0 / (unsigned long long)Q.ngrid);
  const int64_t g = (int64_t)(key0 - (unsigned long long)j0 * Q.ngrid);
  const int is = (int)(g / ((int64_t)Q.nt * Q.np));
  const int it = (int)((g / Q.np) % Q.nt);
  const int ip = (int)(g % Q.np);
  const int inst = Q.inst[j0];
  const double hp = Q.inst_h[inst];
  const double hc = S.inst_h[inst];
  const double Hc = S.inst_H[inst];
  const double kappa = A.inst_kappa[inst];

  // Node geometry of (o, p), as in prop_mfma_kernel.
  for (int i = tid; i < 8 * P; i += blockDim.x) {
    const int o = i / P, p = i - (i / P) * P;
    float u[3];
    float2 rat;
    s_alpha[i] = node_octant_geometry<PS, PA, float>(S, Q, hp, hc, Hc, kappa, is, it, ip, o, p, u, rat);
    s_u[3 * i] = u[0];
    s_u[3 * i + 1] = u[1];
    s_u[3 * i + 2] = u[2];
    s_ratp[2 * i] = rat.x;
    s_ratp[2 * i + 1] = rat.y;
  }
  // Zero the W matrix once: its padding (nodes q >= P, k-steps >= NK) is
  // never written again.
  for (int i = tid; i < P * RS; i += blockDim.x) s_A[i] = 0.f;
  __syncthreads();
  // Distinct child cones of octant o = wave and its nodes grouped by child
  // cone, with wave ballots; lane holds nodes lane and lane + 64.
  {
    const int o = wave;
    const bool has0 = lane < P, has1 = lane + 64 < P;
    const int a0 = has0 ? s_alpha[o * P + lane] : -1;
    const int a1 = has1 ? s_alpha[o * P + lane + 64] : -1;
    bool f0 = has0, f1 = has1;
    int k0 = 0, k1 = 0, na = 0;
    for (;;) {
      const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
      if (m0 == 0ull && m1 == 0ull) break;
      const int lead = m0 ? __shfl(a0, __ffsll((long long)m0) - 1)
                          : __shfl(a1, __ffsll((long long)m1) - 1);
      if (f0 && a0 == lead) { k0 = na; f0 = false; }
      if (f1 && a1 == lead) { k1 = na; f1 = false; }
      if (lane == 0) s_dist[o * P + na] = lead;
      ++na;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
    int base = 0;
    for (int k = 0; k < na; ++k) {
      const unsigned long long m0 = __ballot(has0 && k0 == k), m1 = __ballot(has1 && k1 == k);
      if (has0 && k0 == k) s_rows[o * P + base + __popcll(m0 & lt)] = (unsigned char)lane;
      if (has1 && k1 == k)
        s_rows[o * P + base + __popcll(m0) + __popcll(m1 & lt)] = (unsigned char)(lane + 64);
      if (lane == 0) s_rbeg[o * (P + 1) + k] = base;
      base += __popcll(m0) + __popcll(m1);
    }
    if (lane == 0) {
      s_rbeg[o * (P + 1) + na] = base;
      s_na[o] = na;
    }
  }
  __syncthreads();
  // Lagrange weights and ratios in grouped order.
  for (int i = tid; i < 8 * P; i += blockDim.x) {
    const int o = i / P;
    const int p = s_rows[i];
    const float* u = s_u + 3 * (o * P + p);
    float* L = s_L + i * NW;
    lagrange<PS, float>(u[0], A.cheb.ts, A.cheb.ws, L);
    lagrange<PA, float>(u[1], A.cheb.ta, A.cheb.wa, L + PS);
    lagrange<PA, float>(u[2], A.cheb.ta, A.cheb.wa, L + PS + PA);
    s_rat[2 * i] = s_ratp[2 * (o * P + p)];
    s_rat[2 * i + 1] = s_ratp[2 * (o * P + p) + 1];
  }
  __syncthreads();

  for (int sub = 0; sub * CB < nchunk; ++sub) {
    const int nbk = min(CB, nchunk - sub * CB);
    if (tid < nbk) {
      const int ps = Q.gslot[g0 + (int64_t)sub * CB + tid];
      s_pslot[tid] = ps;
      s_box[tid] = (int)(Q.cone_key[ps] / (unsigned long long)Q.ngrid);
    }
    for (int i = tid; i < B::NCOL * P * 2; i += blockDim.x) s_y[i] = 0.f;
    __syncthreads();
    // Children of the sub-chunk's boxes in octant o = wave, compacted.
    {
      const int o = wave;
      const unsigned long long lt = (1ull << lane) - 1ull;
      int base = 0;
      for (int n0 = 0; n0 < nbk; n0 += 64) {
        const int n = n0 + lane;
        const int kc = n < nbk ? Q.child[8 * (int64_t)s_box[n] + o] : -1;
        const unsigned long long m = __ballot(kc >= 0);
        if (kc >= 0) {
          const int pos = base + __popcll(m & lt);
          s_child[o][pos] = kc;
          s_nl[o][pos] = (unsigned char)n;
        }
        base += __popcll(m);
      }
      if (lane == 0) s_no[o] = base;
    }
    __syncthreads();
    // Child cone slots of octant o into buffer bf.  The octants with
    // children alternate between the two buffers.
    auto lookup = [&](int o, int bf) {
      const int no = s_no[o], na = min(s_na[o], NAMAX);
      for (int i = tid; i < no * na; i += blockDim.x) {
        const int k = i / no, n = i - k * no;
        const int cs = cone_lookup(S, (unsigned long long)s_child[o][n] * S.ngrid +
                                          s_dist[o * P + k]);
        if (cs < 0) atomicOr(A.err, 1);
        s_cs[bf][n * NAMAX + k] = cs;
      }
    };
    int buf = 0;
    {
      int of = 0;
      while (of < 8 && s_no[of] == 0) ++of;
      if (of < 8) lookup(of, 0);
    }
    for (int o = 0; o < 8; ++o) {
      const int no = s_no[o];
      if (no == 0) continue;  // uniform across the block
      const int ncols = no * nrhs;
      const int ntn = (ncols + 15) / 16;
      // W of octant o: one (pos, a, b) per thread, five entries each.
      for (int i = tid; i < P * PS * PA; i += blockDim.x) {
        const int pos = i / (PS * PA), ab = i - (i / (PS * PA)) * (PS * PA);
        const int a = ab / PA, bq = ab - (ab / PA) * PA;
        const float* L = s_L + (o * P + pos) * NW;
        const float lab = L[a] * L[PS + bq];
        float* Ar = s_A + pos * RS;
#pragma unroll
        for (int cq = 0; cq < PA; ++cq) {
          const int q = (a * PA + bq) * PA + cq;
          Ar[B::kgroup(q) * KS + B::kstep(q)] = lab * L[PS + PA + cq];
        }
      }
      // The next octant's slots, into the buffer the previous octant read.
      {
        int o1 = o + 1;
        while (o1 < 8 && s_no[o1] == 0) ++o1;
        if (o1 < 8) lookup(o1, buf ^ 1);
      }
      __syncthreads();
      const int* rbeg = s_rbeg + o * (P + 1);
      int nmt = 0;
      for (int k = 0; k < s_na[o]; ++k) nmt += (rbeg[k + 1] - rbeg[k] + 31) / 32;
      const int nitem = nmt * ntn;
      if (wave < nitem) {
        float br0[B::NK], bi0[B::NK], br1[B::NK], bi1[B::NK];
#define IFGF_BIG_LOAD(IT, LIVE, BR, BI)                                                     \
  big_load_b<PS, PA, MAXR>(S, Vc, A.err, s_cs[buf], s_child[o], s_dist + o * P, rbeg, IT, ntn,  \
                           ncols, nrhs, lane, LIVE, BR, BI)
#define IFGF_BIG_COMP(IT, BR, BI)                                                         \
  big_compute<PS, PA, MAXR>(s_A, s_rat + 2 * o * P, s_rows + o * P, rbeg, s_nl[o], s_y, IT, \
                            ntn, ncols, nrhs, lane, BR, BI)
        // Past the wave's last item the prefetch reads one line that every
        // lane shares, and is not used.
        int item = wave;
        IFGF_BIG_LOAD(item, true, br0, bi0);
        for (;;) {
          const int i1 = item + NWV < nitem ? item + NWV : item;
          IFGF_BIG_LOAD(i1, i1 != item, br1, bi1);
          IFGF_BIG_COMP(item, br0, bi0);
          if (i1 == item) break;
          item = i1;
          const int i2 = item + NWV < nitem ? item + NWV : item;
          IFGF_BIG_LOAD(i2, i2 != item, br0, bi0);
          IFGF_BIG_COMP(item, br1, bi1);
          if (i2 == item) break;
          item = i2;
        }
#undef IFGF_BIG_LOAD
#undef IFGF_BIG_COMP
      }
      buf ^= 1;
      __syncthreads();
    }
    // Write the parent cones of this sub-chunk.
    for (int idx = tid; idx < nbk * nrhs * P; idx += blockDim.x) {
      const int bx = idx / (nrhs * P);
      const int rem = idx - bx * (nrhs * P);
      const int r = rem / P, p = rem - (rem / P) * P;
      float2 v;
      v.x = s_y[2 * ((bx * MAXR + r) * P + p)];
      v.y = s_y[2 * ((bx * MAXR + r) * P + p) + 1];
      Vp[((int64_t)s_pslot[bx] * nrhs + r) * P + p] = v;
    }
    __syncthreads();
  }
}

// Matrix-core propagation for levels where few to some hundred boxes share
// a parent cone index.  A block of NWV waves takes a chunk of up to NWV * WB
// parent boxes sharing (instance, gamma') and accumulates their cones in
// LDS.  Octant by octant the block computes the node geometry (child cone,
// local coordinates, ratio) of the nodes, groups them by child cone and
// compacts the children of its boxes in the octant; the waves then share
// the products
//     C[p][(box, rhs)] = sum_q W[p][q] X[q][(box, rhs)]
// on 16x16x4 MFMA tiles (an N-tile: 16 (child, rhs) columns; an M-tile: up
// to 16 nodes of one child cone), W[p][q] = L_a(u_s) L_b(u_theta) L_c(u_phi)
// formed per tile, adding ratio(p) * C to the accumulators.  The factors
// L_a, L_b, L_c of a row come
// from LDS (several waves: formed once per octant) or are evaluated in
// registers per tile (one wave: the LDS they would take keeps a third wave
// per SIMD resident).
//
// K order.  A k-step is (g, c) with c the phi index of the node; its four
// lane groups kq take four (a, b) pairs: for g < PS the pair (g, kq)
// (kq < min(PA, 4)), for g = PS + e the pair (kq, 4 + e) (kq < PS), other
// slots have weight 0.  A lane's weights are then L_c(c) times L_a(g) L_b(kq)
// or L_a(kq) L_b(4 + e), so it selects one L_a and one L_b value per tile,
// and its B values for each g are PA adjacent nodes of the child cone.
template <int PS, int PA, typename T, int MAXR>
struct SmallProp {
  static constexpr int P = PS * PA * PA;
  static constexpr int PB = PA < 4 ? PA : 4;  // b = kq in the first PS groups
  static constexpr int NE = PA > 4 ? PA - 4 : 0;  // groups with b = 4 + e, a = kq
  static constexpr int NG = PS + NE;
  static constexpr int NK = NG * PA;          // k-steps (g, c)
  static constexpr int NAMAX = 8;             // child cones per octant with a cached slot
  // s_L row: the slot products L_a L_b at kq NG + g, then L_c; 16 bytes.
  static constexpr int LW = (4 * NG + PA + 3) / 4 * 4;
  static_assert(PS <= 4 && PA <= 8, "slot mapping");
  // (a, b) of slot (g, kq), false for a zero slot.
  static __device__ __forceinline__ bool slot_ab(int g, int kq, int& a, int& b) {
    a = g < PS ? g : kq;
    b = g < PS ? kq : 4 + (g - PS);
    return g < PS ? kq < PB : kq < PS;
  }
  // First node index (a PA + b) PA of slot (g, kq), or -1 for a zero slot.
  static __device__ __forceinline__ int slot_row(int g, int kq) {
    int a, b;
    return slot_ab(g, kq, a, b) ? (a * PA + b) * PA : -1;
  }
};

// One Lagrange basis function L_j(u) = w_j prod_{m != j} (u - t_m) for a
// lane-dependent j (a product over all m, no indexed registers).
template <int N, typename T>
__device__ __forceinline__ T lagrange_at(T u, const double* t, int j, T wj) {
  T prod = wj;
#pragma unroll
  for (int m = 0; m < N; ++m) prod *= m == j ? (T)1 : u - (T)t[m];
  return prod;
}

// B values of one lane (column of vp, lane group kq), in k-step order.
template <int PS, int PA, typename T, int MAXR>
__device__ __forceinline__ void small_load_b(const typename C2<T>::type* __restrict__ vp, int kq,
                                             T* br, T* bi) {
  typedef SmallProp<PS, PA, T, MAXR> SP;
  typedef typename C2<T>::type CT;
#pragma unroll
  for (int g = 0; g < SP::NG; ++g) {
    const int q0 = SP::slot_row(g, kq);
    const CT* src = vp + (q0 >= 0 ? q0 : 0);  // zero slot: weight 0
    if constexpr (sizeof(T) == 4) {
      typedef T v4u __attribute__((ext_vector_type(4), aligned(8)));
#pragma unroll
      for (int c = 0; c + 1 < PA; c += 2) {
        const v4u x = *reinterpret_cast<const v4u*>(src + c);
        br[g * PA + c] = x.x;
        bi[g * PA + c] = x.y;
        br[g * PA + c + 1] = x.z;
        bi[g * PA + c + 1] = x.w;
      }
      if constexpr (PA & 1) {
        const CT x = src[PA - 1];
        br[g * PA + PA - 1] = x.x;
        bi[g * PA + PA - 1] = x.y;
      }
    } else {
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        const CT x = src[c];
        br[g * PA + c] = x.x;
        bi[g * PA + c] = x.y;
      }
    }
  }
}

// B values of one lane as in small_load_b, one part of each complex value:
// real parts for part 0, imaginary parts for part 1.
template <int PS, int PA, typename T, int MAXR>
__device__ __forceinline__ void small_load_b1(const typename C2<T>::type* __restrict__ vp, int kq,
                                              int part, T* b) {
  typedef SmallProp<PS, PA, T, MAXR> SP;
  typedef typename C2<T>::type CT;
#pragma unroll
  for (int g = 0; g < SP::NG; ++g) {
    const int q0 = SP::slot_row(g, kq);
    const CT* src = vp + (q0 >= 0 ? q0 : 0);  // zero slot: weight 0
    if constexpr (sizeof(T) == 4) {
      typedef T v4u __attribute__((ext_vector_type(4), aligned(8)));
#pragma unroll
      for (int c = 0; c + 1 < PA; c += 2) {
        const v4u x = *reinterpret_cast<const v4u*>(src + c);
        b[g * PA + c] = part ? x.y : x.x;
        b[g * PA + c + 1] = part ? x.w : x.z;
      }
      if constexpr (PA & 1) {
        const CT x = src[PA - 1];
        b[g * PA + PA - 1] = part ? x.y : x.x;
      }
    } else {
#pragma unroll
      for (int c = 0; c < PA; ++c) b[g * PA + c] = reinterpret_cast<const T*>(src + c)[part];
    }
  }
}

// Three-term BF16 form of the propagation product (an addition beyond the
// paper): each FP32 operand x is split into x_hi = bf16(x) and
// x_lo = bf16(x - x_hi) (round to nearest even), and A B is taken as
// A_lo B_hi + A_hi B_lo + A_hi B_hi on v_mfma_f32_16x16x32_bf16 with FP32
// accumulation; the dropped A_lo B_lo and the rounding of the low parts
// leave a relative error of about 2^-16 per product.  A lane's K values keep
// the k-step order of the FP32 form, eight per instruction (value v = 8 s + i,
// zero from NK on); A and B share the (lane group, element) -> k pairing.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

template <int NK>
struct SplitB {
  static constexpr int NS = (NK + 7) / 8;  // BF16 instructions per product
  bf8v rh[NS], rl[NS], ih[NS], il[NS];    // Re and Im, high and low parts
};

template <int NK>
__device__ __forceinline__ void split_b(const float* br, const float* bi, SplitB<NK>& sb) {
#pragma unroll
  for (int st = 0; st < SplitB<NK>::NS; ++st)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int v = 8 * st + i;
      const float xr = v < NK ? br[v] : 0.f, xi = v < NK ? bi[v] : 0.f;
      const __bf16 hr = (__bf16)xr, hi = (__bf16)xi;
      sb.rh[st][i] = hr;
      sb.rl[st][i] = (__bf16)(xr - (float)hr);
      sb.ih[st][i] = hi;
      sb.il[st][i] = (__bf16)(xi - (float)hi);
    }
}

// One M-tile (rows rb .. rb + rlen - 1 of the octant's grouping, rlen <= 16,
// all of one child cone) times the lane's B values, added with the ratio
// into the accumulators y.  LREG: factors evaluated from s_u (node order)
// instead of read from s_L (grouped order); wak, wbk are the weights of
// L_a(kq), L_b(kq).  SPLIT: the product in three-term BF16 form, B taken
// from sb.
template <int PS, int PA, typename T, int MAXR, bool LREG, bool SPLIT, bool CPLX>
__device__ __forceinline__ void small_tile(const T* s_L, const T* s_u, const ChebConst& cheb,
                                           T wak, T wbk, const typename C2<T>::type* s_ratp,
                                           const unsigned char* s_rows,
                                           typename C2<T>::type* y, int rb, int rlen, int yb,
                                           bool colok, int lane, int part, const T* br,
                                           const T* bi,
                                           const SplitB<SmallProp<PS, PA, T, MAXR>::NK>& sb) {
  typedef SmallProp<PS, PA, T, MAXR> SP;
  typedef typename C2<T>::type CT;
  typedef typename Mfma<T>::v4 V4;
  constexpr int P = SP::P, NG = SP::NG, LW = SP::LW;
  const int kq = lane >> 4;
  const int arow = min(rb + (lane & 15), P - 1);
  // ab[g]: L_a(g) L_b(kq) for g < PS, L_a(kq) L_b(4 + g - PS) above.
  T ab[NG], Lc[PA];
  if constexpr (LREG) {
    T La[PS], Lb4[PA > 4 ? PA - 4 : 1];
    const T* u = s_u + 3 * (int)s_rows[arow];
    const T u0 = u[0], u1 = u[1];
    T lak, lbk;
    lagrange<PS, T>(u0, cheb.ts, cheb.ws, La);
    lagrange<PA, T>(u[2], cheb.ta, cheb.wa, Lc);
    lak = kq < PS ? lagrange_at<PS, T>(u0, cheb.ts, kq, wak) : (T)0;
    lbk = kq < SP::PB ? lagrange_at<PA, T>(u1, cheb.ta, kq, wbk) : (T)0;
#pragma unroll
    for (int e = 0; e < SP::NE; ++e)
      Lb4[e] = lagrange_at<PA, T>(u1, cheb.ta, 4 + e, (T)cheb.wa[4 + e]);
#pragma unroll
    for (int g = 0; g < NG; ++g) ab[g] = g < PS ? La[g] * lbk : lak * Lb4[g < PS ? 0 : g - PS];
  } else {
    const T* L = s_L + arow * LW;
#pragma unroll
    for (int g = 0; g < NG; ++g) ab[g] = L[kq * NG + g];
#pragma unroll
    for (int c = 0; c < PA; ++c) Lc[c] = L[4 * NG + c];
  }
  int pe[4];
  CT rat[4];
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const int mm = Mfma<T>::row(lane, r4);
    pe[r4] = mm < rlen ? (int)s_rows[rb + mm] : -1;
    rat[r4] = s_ratp[pe[r4] >= 0 ? pe[r4] : 0];
  }
  if constexpr (CPLX) {
    // Columns are (child, rhs, part): the lane's B values are the real
    // (part 0) or imaginary (part 1) parts, and its partner lane (col ^ 1)
    // holds the other part of the same complex column.
    V4 acc = {0, 0, 0, 0};
    if constexpr (SPLIT) {
      static_assert(sizeof(T) == 4, "three-term BF16 form of the FP32 product");
      constexpr int NK = SP::NK;
#pragma unroll
      for (int st = 0; st < SplitB<NK>::NS; ++st) {
        bf8v ah, al;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int v = 8 * st + i;
          const float x = v < NK ? ab[v < NK ? v / PA : 0] * Lc[v < NK ? v % PA : 0] : 0.f;
          const __bf16 h = (__bf16)x;
          ah[i] = h;
          al[i] = (__bf16)(x - (float)h);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, sb.rh[st], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.rl[st], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.rh[st], acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int c = 0; c < PA; ++c) acc = Mfma<T>::mma(ab[g] * Lc[c], br[g * PA + c], acc);
    }
    T oth[4];
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) oth[r4] = __shfl_xor(acc[r4], 1);
    if (colok) {
      T* yf = reinterpret_cast<T*>(y);
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        if (pe[r4] >= 0) {
          const T re = part ? oth[r4] : acc[r4], im = part ? acc[r4] : oth[r4];
          const T v = part ? re * rat[r4].y + im * rat[r4].x : re * rat[r4].x - im * rat[r4].y;
          yf[2 * (yb + pe[r4]) + part] += v;
        }
      }
    }
    return;
  }
  V4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  if constexpr (SPLIT) {
    static_assert(sizeof(T) == 4, "three-term BF16 form of the FP32 product");
    constexpr int NK = SP::NK;
#pragma unroll
    for (int st = 0; st < SplitB<NK>::NS; ++st) {
      bf8v ah, al;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int v = 8 * st + i;
        const float x = v < NK ? ab[v < NK ? v / PA : 0] * Lc[v < NK ? v % PA : 0] : 0.f;
        const __bf16 h = (__bf16)x;
        ah[i] = h;
        al[i] = (__bf16)(x - (float)h);
      }
      accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, sb.rh[st], accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, sb.ih[st], acci, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.rl[st], accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.il[st], acci, 0, 0, 0);
      accr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.rh[st], accr, 0, 0, 0);
      acci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, sb.ih[st], acci, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        const T av = ab[g] * Lc[c];
        accr = Mfma<T>::mma(av, br[g * PA + c], accr);
        acci = Mfma<T>::mma(av, bi[g * PA + c], acci);
      }
  }
  if (colok) {
    CT y0[4];
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4)
      if (pe[r4] >= 0) y0[r4] = y[yb + pe[r4]];
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) {
      if (pe[r4] >= 0) {
        CT v;
        v.x = y0[r4].x + accr[r4] * rat[r4].x - acci[r4] * rat[r4].y;
        v.y = y0[r4].y + accr[r4] * rat[r4].y + acci[r4] * rat[r4].x;
        y[yb + pe[r4]] = v;
      }
    }
  }
}

// One M-tile of the one-wave kernel against its (one or two) N-tiles of
// complex-interleaved columns: the Lagrange factors of the lane's row are
// evaluated once, the two products run as interleaved accumulation chains,
// and each N-tile's partner lanes complete the complex ratio multiply as in
// small_tile.
template <int PS, int PA, typename T, int MAXR>
__device__ __forceinline__ void small_tile_cplx2(const T* s_u, const ChebConst& cheb, T wak,
                                                 T wbk, const typename C2<T>::type* s_ratp,
                                                 const unsigned char* s_rows,
                                                 typename C2<T>::type* y, int rb, int rlen,
                                                 int ntn, const int* yb, const bool* colok,
                                                 int lane, int part, const T* br0,
                                                 const T* br1) {
  typedef SmallProp<PS, PA, T, MAXR> SP;
  typedef typename C2<T>::type CT;
  typedef typename Mfma<T>::v4 V4;
  constexpr int P = SP::P, NG = SP::NG;
  const int kq = lane >> 4;
  const int arow = min(rb + (lane & 15), P - 1);
  T ab[NG], Lc[PA];
  {
    T La[PS], Lb4[PA > 4 ? PA - 4 : 1];
    const T* u = s_u + 3 * (int)s_rows[arow];
    const T u0 = u[0], u1 = u[1];
    lagrange<PS, T>(u0, cheb.ts, cheb.ws, La);
    lagrange<PA, T>(u[2], cheb.ta, cheb.wa, Lc);
    const T lak = kq < PS ? lagrange_at<PS, T>(u0, cheb.ts, kq, wak) : (T)0;
    const T lbk = kq < SP::PB ? lagrange_at<PA, T>(u1, cheb.ta, kq, wbk) : (T)0;
#pragma unroll
    for (int e = 0; e < SP::NE; ++e)
      Lb4[e] = lagrange_at<PA, T>(u1, cheb.ta, 4 + e, (T)cheb.wa[4 + e]);
#pragma unroll
    for (int g = 0; g < NG; ++g) ab[g] = g < PS ? La[g] * lbk : lak * Lb4[g < PS ? 0 : g - PS];
  }
  int pe[4];
  CT rat[4];
#pragma unroll
  for (int r4 = 0; r4 < 4; ++r4) {
    const int mm = Mfma<T>::row(lane, r4);
    pe[r4] = mm < rlen ? (int)s_rows[rb + mm] : -1;
    rat[r4] = s_ratp[pe[r4] >= 0 ? pe[r4] : 0];
  }
  V4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  if (ntn > 1) {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int c = 0; c < PA; ++c) {
        const T av = ab[g] * Lc[c];
        acc0 = Mfma<T>::mma(av, br0[g * PA + c], acc0);
        acc1 = Mfma<T>::mma(av, br1[g * PA + c], acc1);
      }
  } else {
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int c = 0; c < PA; ++c) acc0 = Mfma<T>::mma(ab[g] * Lc[c], br0[g * PA + c], acc0);
  }
  T* yf = reinterpret_cast<T*>(y);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t >= ntn) break;  // uniform
    const V4 acc = t ? acc1 : acc0;
    T oth[4];
#pragma unroll
    for (int r4 = 0; r4 < 4; ++r4) oth[r4] = __shfl_xor(acc[r4], 1);
    if (colok[t]) {
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) {
        if (pe[r4] >= 0) {
          const T re = part ? oth[r4] : acc[r4], im = part ? acc[r4] : oth[r4];
          const T v = part ? re * rat[r4].y + im * rat[r4].x : re * rat[r4].x - im * rat[r4].y;
          yf[2 * (yb[t] + pe[r4]) + part] += v;
        }
      }
    }
  }
}

// Box-independent data of one (parent cone index gamma', octant o) of a
// propagation step, in one record (the same layout in LDS and in the
// plan-time table): the number of distinct child cones na and of M-tiles
// nm; the distinct child cones; the nodes grouped by child cone (rows:
// node at grouped position, rbeg: first position of each child cone); the
// M-tiles (child cone, first position); the local coordinates u of every
// node in its child cone; the ratio G(x, x_k)/G(x, x_j) of every node, in
// node order and in grouped order.
template <int P, typename T>
struct OctRec {
  typedef typename C2<T>::type CT;
  static constexpr int kNa = 0, kNm = 4;
  static constexpr int kDist = 16;                                  // int[P]
  static constexpr int kRows = kDist + 4 * P;                       // uchar[P]
  static constexpr int kRbeg = kRows + P;                           // uchar[P + 1]
  static constexpr int kMk = kRbeg + P + 1;                         // uchar[P]
  static constexpr int kMr = kMk + P;                               // uchar[P]
  static constexpr int kU = (kMr + P + 15) / 16 * 16;               // T[3 P]
  static constexpr int kRat = (kU + 3 * P * (int)sizeof(T) + 15) / 16 * 16;  // CT[P]
  static constexpr int kRatg = kRat + P * (int)sizeof(CT);                   // CT[P]
  static constexpr int kSize = (kRatg + P * (int)sizeof(CT) + 15) / 16 * 16;
  unsigned char* b;
  __device__ int& na() const { return *reinterpret_cast<int*>(b + kNa); }
  __device__ int& nm() const { return *reinterpret_cast<int*>(b + kNm); }
  __device__ int* dist() const { return reinterpret_cast<int*>(b + kDist); }
  __device__ unsigned char* rows() const { return b + kRows; }
  __device__ unsigned char* rbeg() const { return b + kRbeg; }
  __device__ unsigned char* mk() const { return b + kMk; }
  __device__ unsigned char* mr() const { return b + kMr; }
  __device__ T* u() const { return reinterpret_cast<T*>(b + kU); }
  __device__ CT* ratp() const { return reinterpret_cast<CT*>(b + kRat); }
  __device__ CT* ratg() const { return reinterpret_cast<CT*>(b + kRatg); }  // grouped order
};

// node_octant_geometry for nodes p = t0, t0 + stride, ... into a record.
template <int PS, int PA, typename T>
__device__ __forceinline__ void octant_geometry(const StepDev& S, const StepDev& Q, double hp,
                                                double hc, double Hc, double kappa, int is,
                                                int it, int ip, int o, int t0, int stride,
                                                int* s_alpha, OctRec<PS * PA * PA, T> R) {
  constexpr int P = PS * PA * PA;
  for (int p = t0; p < P; p += stride) {
    T u[3];
    s_alpha[p] = node_octant_geometry<PS, PA, T>(S, Q, hp, hc, Hc, kappa, is, it, ip, o, p, u,
                                                 R.ratp()[p]);
    R.u()[3 * p] = u[0];
    R.u()[3 * p + 1] = u[1];
    R.u()[3 * p + 2] = u[2];
  }
}

// Distinct child cones, the nodes grouped by child cone and the M-tiles of
// every child cone, from alpha(p) (one wave, ballots; lane holds nodes lane
// and lane + 64).
template <int P, typename T>
__device__ __forceinline__ void octant_grouping(const int* s_alpha, int lane,
                                                OctRec<P, T> R) {
  const unsigned long long lt = (1ull << lane) - 1ull;
  const bool has0 = lane < P, has1 = lane + 64 < P;
  const int a0 = has0 ? s_alpha[lane] : -1;
  const int a1 = has1 ? s_alpha[lane + 64] : -1;
  bool f0 = has0, f1 = has1;
  int k0 = 0, k1 = 0, na = 0;
  int* dist = R.dist();
  for (;;) {
    const unsigned long long m0 = __ballot(f0), m1 = __ballot(f1);
    if (m0 == 0ull && m1 == 0ull) break;
    const int lead = m0 ? __shfl(a0, __ffsll((long long)m0) - 1)
                        : __shfl(a1, __ffsll((long long)m1) - 1);
    if (f0 && a0 == lead) { k0 = na; f0 = false; }
    if (f1 && a1 == lead) { k1 = na; f1 = false; }
    if (lane == 0) dist[na] = lead;
    ++na;
  }
  unsigned char* rows = R.rows();
  int base = 0, nm = 0;
  for (int k = 0; k < na; ++k) {
    const unsigned long long m0 = __ballot(has0 && k0 == k), m1 = __ballot(has1 && k1 == k);
    if (has0 && k0 == k) rows[base + __popcll(m0 & lt)] = (unsigned char)lane;
    if (has1 && k1 == k) rows[base + __popcll(m0) + __popcll(m1 & lt)] = (unsigned char)(lane + 64);
    const int rlen = __popcll(m0) + __popcll(m1);
    const int ntk = (rlen + 15) >> 4;
    if (lane < ntk) {
      R.mk()[nm + lane] = (unsigned char)k;
      R.mr()[nm + lane] = (unsigned char)(base + 16 * lane);
    }
    if (lane == 0) R.rbeg()[k] = base;
    base += rlen;
    nm += ntk;
  }
  if (lane == 0) {
    R.rbeg()[na] = base;
    R.na() = na;
    R.nm() = nm;
  }
  // The ratios in grouped order (LDS operations of one wave complete in
  // order, so the rows written above are visible here).
  for (int pos = lane; pos < P; pos += 64) R.ratg()[pos] = R.ratp()[rows[pos]];
}

// Plan-time table of a propagation step: one record per (group, octant),
// a group being the relevant parent cones sharing (instance, gamma').  One
// wave per record.
template <int PS, int PA, typename T>
__global__ void __launch_bounds__(64) prop_table_kernel(ApplyArgs A, int l) {
  typedef OctRec<PS * PA * PA, T> R;
  constexpr int P = PS * PA * PA;
  __shared__ __align__(16) unsigned char s_rec[R::kSize];
  __shared__ int s_alpha[P];
  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  const int64_t gi = blockIdx.x >> 3;
  const int o = blockIdx.x & 7;
  const int lane = threadIdx.x;
  const unsigned long long key0 = Q.cone_key[Q.gslot[Q.group_first[gi]]];
  const int64_t j0 = (int64_t)(key0 / (unsigned long long)Q.ngrid);
  const int64_t g = (int64_t)(key0 - (unsigned long long)j0 * Q.ngrid);
  const int is = (int)(g / ((int64_t)Q.nt * Q.np));
  const int it = (int)((g / Q.np) % Q.nt);
  const int ip = (int)(g % Q.np);
  const int inst = Q.inst[j0];
  R rec{s_rec};
  octant_geometry<PS, PA, T>(S, Q, Q.inst_h[inst], S.inst_h[inst], S.inst_H[inst],
                             A.inst_kappa[inst], is, it, ip, o, lane, 64, s_alpha, rec);
  __syncthreads();
  octant_grouping<P, T>(s_alpha, lane, rec);
  __syncthreads();
  const uint4* src = reinterpret_cast<const uint4*>(s_rec);
  uint4* dst = reinterpret_cast<uint4*>(Q.prop_table + (int64_t)blockIdx.x * R::kSize);
  for (int i = lane; i < R::kSize / 16; i += 64) dst[i] = src[i];
}

// The children of the block's boxes are compacted per octant across the
// whole block, so an N-tile holds 16 (child, rhs) columns of any of its
// waves' boxes; the octant's work items (N-tile, M-tile) are cut into NWV
// contiguous ranges, one per wave.  Within an octant every (box, node) is
// written by exactly one item (M-tiles of different child cones hold
// different nodes), so the block-wide accumulators need no atomics.
static constexpr int kXcdRun = 256;  // chunks per XCD turn (prop_small_kernel)

template <int PS, int PA, typename T, int MAXR, int NWV, bool SPLIT, int BPW = kTaskBoxes>
__global__ void __launch_bounds__(64 * NWV, sizeof(T) == 4 ? (BPW < kTaskBoxes ? 4 : 3) : 2)
prop_small_kernel(ApplyArgs A, int l, const typename C2<T>::type* __restrict__ Vc,
                  typename C2<T>::type* __restrict__ Vp) {
  typedef SmallProp<PS, PA, T, MAXR> SP;
  typedef typename C2<T>::type CT;
  constexpr int P = SP::P, NAMAX = SP::NAMAX, LW = SP::LW;
  constexpr int NB = NWV * (BPW / MAXR);    // boxes per block
  constexpr bool LREG = NWV == 1;           // factors in registers (one wave)
  // One wave: (child, rhs, part) columns, 8 complex columns per N-tile (its
  // chunks hold few children per octant); several waves: (child, rhs)
  // columns with the real and imaginary parts in separate products.
  constexpr bool CPLX = NWV == 1;

  static_assert(P <= 128, "two nodes per lane");
  static_assert(NB <= 64, "one lane per box");
  typedef OctRec<P, T> Rec;
  // Shared per octant: the octant's record (computed, or copied from the
  // step's plan-time table), the child cone of every node while it is being
  // computed, and the factors in grouped order.
  __shared__ __align__(16) T s_L[LREG ? 1 : P * LW];  // factors at grouped position pos
  __shared__ __align__(16) unsigned char s_rec[Rec::kSize];
  __shared__ int s_alpha[P];                // child cone of node p
  const Rec rec{s_rec};
  const T* const s_u = rec.u();             // local coordinates of node p
  const CT* const s_ratp = rec.ratp();      // ratio of node p
  const unsigned char* const s_rows = rec.rows();  // node p at pos
  const unsigned char* const s_rbeg = rec.rbeg();  // first pos of each child cone
  const int* const s_dist = rec.dist();     // distinct child cones
  const unsigned char* const s_mk = rec.mk();  // M-tile j: child cone, first pos
  const unsigned char* const s_mr = rec.mr();
  // Per block.
  __shared__ CT s_y[NB * MAXR * P];
  __shared__ int s_slot[NB];
  __shared__ int s_ch[8][NB];               // children per octant, compacted
  __shared__ unsigned char s_nl[8][NB];     // their box index in the chunk
  __shared__ unsigned char s_no[8];         // children per octant
  __shared__ int s_cs[NB * NAMAX];          // child cone slots of the current octant

  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nrhs = A.nrhs;
  constexpr bool LEAN = NWV > 1 && BPW < kTaskBoxes;
  const int64_t* cstart = NWV == 1 ? Q.schunk_start : LEAN ? Q.lchunk_start : Q.mchunk_start;
  const int* clen = NWV == 1 ? Q.schunk_len : LEAN ? Q.lchunk_len : Q.mchunk_len;
  // XCD-aware chunk order: workgroups are dispatched round-robin to the eight
  // XCDs (each with its own L2), so each XCD takes runs of kXcdRun
  // consecutive chunks of the dispatch order, in turn; the chunks that read
  // the same child cones then share an L2 (37% less fetched at the
  // 321k-point sphere, at the same time).  A bijection on [0, gridDim.x):
  // the blocks past the last whole turn keep their index.
  const int bid = [] {
    const int n = (int)gridDim.x, b = (int)blockIdx.x;
    const int full = n / (8 * kXcdRun) * (8 * kXcdRun);
    if (b >= full) return b;
    const int x = b % 8, i = b / 8;
    return ((i / kXcdRun) * 8 + x) * kXcdRun + i % kXcdRun;
  }();
  const int64_t g0 = cstart[bid];
  const int nb = clen[bid];          // boxes of this chunk, <= NB
  // The step's table of octant records, and this chunk's group in it.
  const unsigned char* const table =
      Q.prop_table ? Q.prop_table +
                         (int64_t)(NWV == 1 ? Q.schunk_group
                                   : LEAN   ? Q.lchunk_group
                                            : Q.mchunk_group)[bid] * 8 *
                             Rec::kSize
                   : nullptr;
  const unsigned long long key0 = Q.cone_key[Q.gslot[g0]];
  const int64_t j0 = (int64_t)(key0 / (unsigned long long)Q.ngrid);
  const int64_t g = (int64_t)(key0 - (unsigned long long)j0 * Q.ngrid);
  const int is = (int)(g / ((int64_t)Q.nt * Q.np));
  const int it = (int)((g / Q.np) % Q.nt);
  const int ip = (int)(g % Q.np);
  const int inst = Q.inst[j0];
  const double hp = Q.inst_h[inst];
  const double hc = S.inst_h[inst];
  const double Hc = S.inst_H[inst];
  const double kappa = A.inst_kappa[inst];
  const unsigned long long lt = (1ull << lane) - 1ull;

  // The chunk's boxes and their children, compacted per octant (wave 0).
  if (wave == 0) {
    int box = 0;
    if (lane < nb) {
      const int slot = Q.gslot[g0 + lane];
      s_slot[lane] = slot;
      box = (int)(Q.cone_key[slot] / (unsigned long long)Q.ngrid);
    }
    int ch[8];  // all eight loads in flight before the first ballot
#pragma unroll
    for (int o = 0; o < 8; ++o) ch[o] = lane < nb ? Q.child[8 * (int64_t)box + o] : -1;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const unsigned long long m = __ballot(ch[o] >= 0);
      if (ch[o] >= 0) {
        const int pos = __popcll(m & lt);
        s_ch[o][pos] = ch[o];
        s_nl[o][pos] = (unsigned char)lane;
      }
      if (lane == 0) s_no[o] = (unsigned char)__popcll(m);
    }
  }
  for (int i = tid; i < NB * MAXR * P; i += 64 * NWV) s_y[i] = CT{(T)0, (T)0};
  __syncthreads();

  const int col = lane & 15, kq = lane >> 4;
  const T wak = kq < PS ? (T)A.cheb.ws[kq] : (T)0;
  const T wbk = kq < SP::PB ? (T)A.cheb.wa[kq] : (T)0;
  bool miss = false;  // a cone look-up missed (reported once, at the end)
#pragma unroll 1
  for (int o = 0; o < 8; ++o) {
    const int no = s_no[o];
    if (no == 0) continue;  // uniform across the block
    if (table) {
      // The octant's record from the plan-time table.
      const uint4* src = reinterpret_cast<const uint4*>(table + o * Rec::kSize);
      uint4* dst = reinterpret_cast<uint4*>(s_rec);
      for (int i = tid; i < Rec::kSize / 16; i += 64 * NWV) dst[i] = src[i];
      __syncthreads();
    } else {
      octant_geometry<PS, PA, T>(S, Q, hp, hc, Hc, kappa, is, it, ip, o, tid, 64 * NWV, s_alpha,
                                 rec);
      __syncthreads();
      if (wave == 0) octant_grouping<P, T>(s_alpha, lane, rec);
      __syncthreads();
    }
    const int na = rec.na(), nm = rec.nm();
    // Factors in grouped order (several waves); child cone slots of the
    // block's children.
    if constexpr (!LREG) {
      for (int pos = tid; pos < P; pos += 64 * NWV) {
        const int p = s_rows[pos];
        T La[PS], Lb[PA], Lc[PA];
        lagrange<PS, T>(s_u[3 * p], A.cheb.ts, A.cheb.ws, La);
        lagrange<PA, T>(s_u[3 * p + 1], A.cheb.ta, A.cheb.wa, Lb);
        lagrange<PA, T>(s_u[3 * p + 2], A.cheb.ta, A.cheb.wa, Lc);
        T* L = s_L + pos * LW;
#pragma unroll
        for (int gg = 0; gg < SP::NG; ++gg)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            int a, b;
            const bool ok = SP::slot_ab(gg, j, a, b);
            L[j * SP::NG + gg] = ok ? La[a] * Lb[b] : (T)0;
          }
#pragma unroll
        for (int c = 0; c < PA; ++c) L[4 * SP::NG + c] = Lc[c];
      }
    }
    {
      const int nac = min(na, NAMAX);
      for (int e = tid; e < no * nac; e += 64 * NWV) {
        const int k = e / no, n = e - k * no;
        const int cs = cone_lookup(S, (unsigned long long)s_ch[o][n] * S.ngrid + s_dist[k]);
        miss |= cs < 0;
        s_cs[n * NAMAX + k] = cs;
      }
    }
    __syncthreads();
    const int ncols = no * nrhs;  // complex columns (child, rhs)
    if constexpr (NWV == 1 && !SPLIT) {
      // One wave: at most 16 complex columns (a box has one child per
      // octant), so at most two N-tiles.  Per child cone the B values of
      // both are loaded once, and each M-tile's factors serve both.
      const int ntn = (ncols + 7) >> 3;
      int n0c[2], rc[2], ybc[2];
      bool okc[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int c = t * 8 + (col >> 1);
        okc[t] = c < ncols;
        n0c[t] = !okc[t] ? 0 : MAXR == 1 ? c : c / nrhs;
        rc[t] = !okc[t] || MAXR == 1 ? 0 : c - n0c[t] * nrhs;
        ybc[t] = okc[t] ? ((int)s_nl[o][n0c[t]] * MAXR + rc[t]) * P : 0;
      }
      const int part = col & 1;
      for (int k = 0; k < na; ++k) {
        T b0[SP::NK], b1[SP::NK];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (t < ntn) {
            int cs;
            if (k < NAMAX) {
              cs = s_cs[n0c[t] * NAMAX + k];
            } else {
              cs = cone_lookup(S, (unsigned long long)s_ch[o][n0c[t]] * S.ngrid + s_dist[k]);
              miss |= cs < 0;
            }
            const CT* vsrc = Vc + ((int64_t)(cs >= 0 ? cs : 0) * nrhs + rc[t]) * P;
            small_load_b1<PS, PA, T, MAXR>(vsrc, kq, part, t ? b1 : b0);
          }
        }
        for (int rb = s_rbeg[k]; rb < s_rbeg[k + 1]; rb += 16)
          small_tile_cplx2<PS, PA, T, MAXR>(s_u, A.cheb, wak, wbk, s_ratp, s_rows, s_y, rb,
                                            min(16, s_rbeg[k + 1] - rb), ntn, ybc, okc, lane,
                                            part, b0, b1);
      }
    } else {
      // Work items (N-tile nt, M-tile j), nt major; wave w takes a contiguous
      // range and walks it unit by unit, a unit being the M-tiles of one
      // (nt, child cone k) in the range, with one B load per unit.
      const int nit = (CPLX ? (ncols + 7) >> 3 : (ncols + 15) >> 4) * nm;
      const int i0 = (int)(((int64_t)nit * wave) / NWV), i1 = (int)(((int64_t)nit * (wave + 1)) / NWV);
      int nt = i0 / nm, k = 0, rb = 0, rend = 0;
      if (i0 < i1) {
        if constexpr (NWV > 1) {
          const int j = i0 - nt * nm;
          k = s_mk[j];
          rb = s_mr[j];
        }
        rend = s_rbeg[k + 1];
      }
      int item = i0;
      while (item < i1) {
        const int part = CPLX ? col & 1 : 0;
        const int c = CPLX ? nt * 8 + (col >> 1) : nt * 16 + col;
        const bool colok = c < ncols;
        const int n0 = !colok ? 0 : MAXR == 1 ? c : c / nrhs;
        const int r = !colok || MAXR == 1 ? 0 : c - n0 * nrhs;
        const int yb = colok ? ((int)s_nl[o][n0] * MAXR + r) * P : 0;
        int cs;
        if (k < NAMAX) {
          cs = s_cs[n0 * NAMAX + k];
        } else {
          cs = cone_lookup(S, (unsigned long long)s_ch[o][n0] * S.ngrid + s_dist[k]);
          miss |= cs < 0;
        }
        T br[SP::NK], bi[CPLX ? 1 : SP::NK];
        const CT* vsrc = Vc + ((int64_t)(cs >= 0 ? cs : 0) * nrhs + r) * P;
        if constexpr (CPLX)
          small_load_b1<PS, PA, T, MAXR>(vsrc, kq, part, br);
        else
          small_load_b<PS, PA, T, MAXR>(vsrc, kq, br, bi);
        SplitB<SP::NK> sb;
        if constexpr (SPLIT) split_b<SP::NK>((const float*)br, (const float*)(CPLX ? br : bi), sb);
        do {
          small_tile<PS, PA, T, MAXR, LREG, SPLIT, CPLX>(s_L, s_u, A.cheb, wak, wbk, s_ratp, s_rows,
                                                         s_y, rb, min(16, rend - rb), yb, colok,
                                                         lane, part, br, bi, sb);
          ++item;
          rb += 16;
        } while (item < i1 && rb < rend);
        if (rb >= rend) {  // next child cone, or the first of the next N-tile
          if (++k == na) {
            k = 0;
            ++nt;
          }
          rb = s_rbeg[k];
          rend = s_rbeg[k + 1];
        }
      }
    }
    __syncthreads();
  }
  if (miss) atomicOr(A.err, 1);
  // Write the parent cones of the chunk's boxes.
  for (int i = tid; i < nb * nrhs * P; i += 64 * NWV) {
    const int n = i / (nrhs * P);
    const int rem = i - n * (nrhs * P);
    const int r = rem / P, p = rem - (rem / P) * P;
    Vp[((int64_t)s_slot[n] * nrhs + r) * P + p] = s_y[(n * MAXR + r) * P + p];
  }
}

// ---------------------------------------------------------------------------
// Plan-time kernels: relevant cone segments.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void hash_insert(unsigned long long* tab,
                                            unsigned long long mask,
                                            unsigned long long key,
                                            unsigned int* count,
                                            int* overflow) {
  // Bounded probing: a (nearly) full table reports overflow and the planner
  // retries with a larger one, so every insert terminates.
  unsigned long long h = hmix(key) & mask;
  for (unsigned long long probe = 0; probe <= mask && probe < 4096; ++probe) {
    unsigned long long k = __atomic_load_n(&tab[h], __ATOMIC_RELAXED);
    if (k == key) return;
    if (k == kEmptyKey) {
      unsigned long long prev = atomicCAS(&tab[h], kEmptyKey, key);
      if (prev == kEmptyKey) {
        atomicAdd(count, 1u);
        return;
      }
      if (prev == key) return;
    }
    h = (h + 1) & mask;
  }
  atomicOr(overflow, 1);
}

// Insert the cone containing the point with coordinates q, plus the
// adjacent cones when q lies within `margin` (in cone widths) of a cone
// boundary, so that look-ups computed along a different FP64 path land in a
// relevant cone.  phi is periodic.
__device__ __forceinline__ void mark_cone(const StepDev& S, int64_t box,
                                          const double q[3], MarkArgs M) {
  int n[3] = {S.ns, S.nt, S.np};
  int cand[3][3];
  int nc[3];
  for (int d = 0; d < 3; ++d) {
    double u;
    int i = cone_index(q[d], n[d], u);
    double f = 0.5 * (u + 1.0);
    nc[d] = 0;
    cand[d][nc[d]++] = i;
    if (f < M.margin) {
      if (i > 0) cand[d][nc[d]++] = i - 1;
      else if (d == 2 && n[d] > 1) cand[d][nc[d]++] = n[d] - 1;
    }
    if (f > 1.0 - M.margin) {
      if (i < n[d] - 1) cand[d][nc[d]++] = i + 1;
      else if (d == 2 && n[d] > 1) cand[d][nc[d]++] = 0;
    }
  }
  for (int x = 0; x < nc[0]; ++x)
    for (int y = 0; y < nc[1]; ++y)
      for (int z = 0; z < nc[2]; ++z) {
        unsigned long long key = (unsigned long long)box * S.ngrid +
                                 ((unsigned long long)cand[0][x] * S.nt + cand[1][y]) * S.np +
                                 cand[2][z];
        hash_insert(M.tab, M.mask, key, M.count, M.overflow);
      }
}

// Cones of the cousin boxes containing each point: thread per point x, loop
// over the cousins B_k of its box at this step (M^d(x) = M B^d(x)).
__global__ void mark_cousin_kernel(ApplyArgs A, int l, MarkArgs M) {
  int64_t i = gtid();
  if (i >= A.n) return;
  const StepDev& S = A.step[l];
  int b = S.pt_box[i];
  if (b < 0) return;
  double h = S.inst_h[S.inst[b]];
  double xi = A.x[i], yi = A.y[i], zi = A.z[i];
  for (int64_t j = S.cous_begin[b]; j < S.cous_begin[b + 1]; ++j) {
    int k = S.cous[j];
    double y0, y1, y2;
    {
      IFGF_NO_CONTRACT
      y0 = xi - S.center[3 * k];
      y1 = yi - S.center[3 * k + 1];
      y2 = zi - S.center[3 * k + 2];
    }
    ConeCoord c = cone_coord(S, h, y0, y1, y2);
    mark_cone(S, k, c.q, M);
  }
}

// Cones of the children containing each node of a relevant parent cone.
template <int PS, int PA>
__global__ void mark_parent_kernel(ApplyArgs A, int l, MarkArgs M) {
  constexpr int P = PS * PA * PA;
  const StepDev& S = A.step[l];
  const StepDev& Q = A.step[l + 1];
  int64_t t = gtid();
  if (t >= Q.ncones * P) return;
  int64_t slot = t / P;
  int p = (int)(t - slot * P);
  unsigned long long key = Q.cone_key[slot];
  int64_t j = (int64_t)(key / (unsigned long long)Q.ngrid);
  int64_t g = (int64_t)(key - (unsigned long long)j * Q.ngrid);
  int is = (int)(g / ((int64_t)Q.nt * Q.np));
  int it = (int)((g / Q.np) % Q.nt);
  int ip = (int)(g % Q.np);
  int a = p / (PA * PA), bb = (p / PA) % PA, cc = p % PA;
  int inst = Q.inst[j];
  double hp = Q.inst_h[inst];
  double hc = S.inst_h[inst];
  double yp[3];
  node_offset<PS, PA>(Q, hp, is, it, ip, a, bb, cc, yp);
  double x0, x1, x2;
  {
    IFGF_NO_CONTRACT
    x0 = Q.center[3 * j] + yp[0];
    x1 = Q.center[3 * j + 1] + yp[1];
    x2 = Q.center[3 * j + 2] + yp[2];
  }
  for (int o = 0; o < 8; ++o) {
    int k = Q.child[8 * j + o];
    if (k < 0) continue;
    double y0, y1, y2;
    {
      IFGF_NO_CONTRACT
      y0 = x0 - S.center[3 * k];
      y1 = x1 - S.center[3 * k + 1];
      y2 = x2 - S.center[3 * k + 2];
    }
    ConeCoord c = cone_coord(S, hc, y0, y1, y2);
    mark_cone(S, k, c.q, M);
  }
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n,
                                unsigned long long v) {
  int64_t t = gtid();
  if (t < n) p[t] = v;
}

__global__ void fill_i32_kernel(int* p, int64_t n, int v) {
  int64_t t = gtid();
  if (t < n) p[t] = v;
}

// Dense look-up table: table[box * ngrid + gamma] = slot.
__global__ void scatter_table_kernel(const unsigned long long* __restrict__ keys,
                                     int64_t n, int* table) {
  int64_t t = gtid();
  if (t < n) table[keys[t]] = (int)t;
}

__global__ void compact_keys_kernel(const unsigned long long* __restrict__ tab,
                                    int64_t cap, unsigned long long* out,
                                    unsigned int* counter) {
  int64_t t = gtid();
  if (t >= cap) return;
  unsigned long long k = tab[t];
  if (k != kEmptyKey) out[atomicAdd(counter, 1u)] = k;
}

// Final table: key -> slot (index in the sorted key array).
__global__ void build_lookup_kernel(const unsigned long long* __restrict__ keys,
                                    int64_t n, unsigned long long* tab,
                                    int* val, unsigned long long mask,
                                    int* overflow) {
  int64_t t = gtid();
  if (t >= n) return;
  unsigned long long key = keys[t];
  unsigned long long h = hmix(key) & mask;
  for (unsigned long long probe = 0; probe <= mask; ++probe) {
    unsigned long long prev = atomicCAS(&tab[h], kEmptyKey, key);
    if (prev == kEmptyKey || prev == key) {
      val[h] = (int)t;
      return;
    }
    h = (h + 1) & mask;
  }
  atomicOr(overflow, 1);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

// Grid covering n threads in blocks of bs: at most 2^22 blocks in x (2^30
// work-items), the rest in y; threads past n exit in the kernels.
static inline dim3 nblk(int64_t n, int bs) {
  const int64_t b = std::max<int64_t>(1, (n + bs - 1) / bs);
  const int64_t bx = std::min<int64_t>(b, int64_t(1) << 22);
  return dim3((unsigned)bx, (unsigned)((b + bx - 1) / bx), 1);
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n,
                           unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  fill_u64_kernel<<<nblk(n, 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_mark(const ApplyArgs& A, int l, int ps, int pa,
                       const MarkArgs& M, hipStream_t st) {
  if (A.n > 0) mark_cousin_kernel<<<nblk(A.n, 256), 256, 0, st>>>(A, l, M);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (l + 1 < A.n_steps && A.step_host[l + 1].ncones > 0) {
    int64_t work = A.step_host[l + 1].ncones * (int64_t)(ps * pa * pa);
#define IFGF_MARK(PS_, PA_)                                                   \
  if (ps == PS_ && pa == PA_)                                                 \
    mark_parent_kernel<PS_, PA_><<<nblk(work, 256), 256, 0, st>>>(A, l, M);
    IFGF_MARK(3, 5) else IFGF_MARK(2, 3) else IFGF_MARK(5, 7) else return hipErrorInvalidValue;
#undef IFGF_MARK
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  fill_i32_kernel<<<nblk(n, 256), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_scatter_table(const unsigned long long* keys, int64_t n,
                                int* table, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  scatter_table_kernel<<<nblk(n, 256), 256, 0, st>>>(keys, n, table);
  return hipGetLastError();
}

hipError_t launch_compact(const unsigned long long* tab, int64_t cap,
                          unsigned long long* out, unsigned int* counter,
                          hipStream_t st) {
  compact_keys_kernel<<<nblk(cap, 256), 256, 0, st>>>(tab, cap, out, counter);
  return hipGetLastError();
}

hipError_t launch_build_lookup(const unsigned long long* keys, int64_t n,
                               unsigned long long* tab, int* val,
                               unsigned long long mask, int* overflow,
                               hipStream_t st) {
  if (n <= 0) return hipSuccess;
  build_lookup_kernel<<<nblk(n, 256), 256, 0, st>>>(keys, n, tab, val, mask, overflow);
  return hipGetLastError();
}

// Group keys of a level's cones: instance * grid + gamma, with the slot as
// the value to sort.
__global__ void group_key_kernel(const unsigned long long* __restrict__ keys, int64_t n,
                                 unsigned long long ng, const int* __restrict__ inst,
                                 unsigned long long* __restrict__ gk, int* __restrict__ idx) {
  const int64_t t = gtid();
  if (t >= n) return;
  const unsigned long long k = keys[t], b = k / ng;
  gk[t] = (unsigned long long)inst[b] * ng + (k - b * ng);
  idx[t] = (int)t;
}

hipError_t launch_group_keys(const unsigned long long* keys, int64_t n, unsigned long long ng,
                             const int* inst, unsigned long long* gk, int* idx,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  group_key_kernel<<<nblk(n, 256), 256, 0, st>>>(keys, n, ng, inst, gk, idx);
  return hipGetLastError();
}

// Stable radix sort of (64-bit key, int) pairs (rocPRIM): equal keys keep
// their input order.  With scratch == nullptr only the scratch size is
// returned.
hipError_t sort_pairs(const unsigned long long* keys_in, unsigned long long* keys_out,
                      const int* vals_in, int* vals_out, int64_t n, int end_bit, void* scratch,
                      size_t* scratch_bytes, hipStream_t st) {
  return rocprim::radix_sort_pairs(scratch, *scratch_bytes, keys_in, keys_out, vals_in,
                                   vals_out, (size_t)n, 0u, (unsigned)end_bit, st);
}

// Radix sort of 64-bit keys (rocPRIM).  With scratch == nullptr only the
// scratch size is returned.
hipError_t sort_keys(unsigned long long* keys, unsigned long long* tmp,
                     int64_t n, int end_bit, void* scratch,
                     size_t* scratch_bytes, hipStream_t st) {
  hipError_t e = rocprim::radix_sort_keys(scratch, *scratch_bytes, keys, tmp,
                                          (size_t)n, 0u, (unsigned)end_bit, st);
  if (e != hipSuccess || scratch == nullptr) return e;
  return hipMemcpyAsync(keys, tmp, sizeof(unsigned long long) * n,
                        hipMemcpyDeviceToDevice, st);
}

// Launch with optional event timing of the launch.
#define IFGF_TIMED(stage, launch)                                  \
  do {                                                             \
    if (prof) {                                                    \
      hipError_t pe_ = prof->begin(stage, st);                     \
      if (pe_ != hipSuccess) return pe_;                           \
    }                                                              \
    launch;                                                        \
    if (prof) {                                                    \
      hipError_t pe_ = prof->end(st);                              \
      if (pe_ != hipSuccess) return pe_;                           \
    }                                                              \
  } while (0)

int small_chunk_boxes(int nrhs, int waves, int per_wave) {
  return waves * (per_wave / (nrhs <= 1 ? 1 : kMaxRhs));
}

int chunk_boxes(int precision, int nrhs) {
  const int maxr = nrhs <= 1 ? 1 : kMaxRhs;
  return kSubChunks *
         (precision == 0 ? ChunkCols<double, 1>::boxes : ChunkCols<float, 1>::boxes) / maxr;
}

// The grouped (matrix-core) propagation of one level: 512-thread blocks in
// FP32, 256-thread blocks in FP64 (whose operands do not fit the former's
// LDS layout).
// The per-node propagation: one thread per (relevant parent cone, node),
// child cones staged in LDS per wave.
template <int PS, int PA, typename T, int MAXR>
static void launch_prop_node(const ApplyArgs& A, int l, const typename C2<T>::type* Vc,
                             typename C2<T>::type* Vp, int64_t ncones, hipStream_t st) {
  constexpr int P = PS * PA * PA;
  prop_node_kernel<PS, PA, T, MAXR><<<nblk(ncones * P, 64), 64, 0, st>>>(A, l, Vc, Vp);
}

template <int PS, int PA, typename T, int MAXR>
static void launch_grouped(const ApplyArgs& A, int l, const typename C2<T>::type* Vc,
                           typename C2<T>::type* Vp, int64_t nchunks, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    prop_big_kernel<PS, PA, MAXR><<<(unsigned)nchunks, 512, 0, st>>>(A, l, Vc, Vp);
  } else {
    prop_mfma_kernel<PS, PA, T, MAXR><<<(unsigned)nchunks, kMfmaThreads, 0, st>>>(A, l, Vc, Vp);
  }
}

template <int PS, int PA, typename T, int MAXR, bool SPLIT>
static hipError_t apply_impl(const ApplyArgs& A, const void* dens_user,
                             void* out_user, hipStream_t st, Profiler* prof) {
  typedef typename C2<T>::type CT;
  constexpr int P = PS * PA * PA;
  const int64_t nr = A.n * A.nrhs;
  CT* ds = (CT*)A.dens_sorted;
  CT* os = (CT*)A.out_sorted;
  IFGF_TIMED(0, (perm_in_kernel<T><<<nblk(nr, 256), 256, 0, st>>>(
                    (const CT*)dens_user, ds, A.perm, A.n, A.nrhs)));
  if (A.stages & 1)
    IFGF_TIMED(1, (near_field_kernel<T, MAXR><<<nblk(A.n, 256), 256, 0, st>>>(A, os)));
  else
    IFGF_TIMED(1, (zero_kernel<T><<<nblk(nr, 256), 256, 0, st>>>(os, nr)));
  if (A.stages & 2) {
    CT* Vcur = (CT*)A.vbuf[0];
    CT* Vnext = (CT*)A.vbuf[1];
    const StepDev& S0 = A.step_host[0];
    if (S0.ncones > 0)
      IFGF_TIMED(2, (leaf_eval_kernel<PS, PA, T, MAXR>
                     <<<nblk(S0.ncones * P, 256), 256, 0, st>>>(A, Vcur)));
    for (int l = 0; l < A.n_steps; ++l) {
      if (A.step_host[l].ncones > 0)
        IFGF_TIMED(3, (interp_kernel<PS, PA, T, MAXR><<<nblk(A.n, 64), 64 * kInterpParts, 0,
                                                        st>>>(A, l, Vcur, os)));
      if (l + 1 < A.n_steps && A.step_host[l + 1].ncones > 0) {
        const StepDev& Qh = A.step_host[l + 1];
        bool done = false;
        if constexpr (P <= kMfmaMaxP) {
          if (Qh.prop_grouped == kPropGrouped) {
            IFGF_TIMED(6, (launch_grouped<PS, PA, T, MAXR>(A, l, Vcur, Vnext, Qh.nchunks, st)));
            done = true;
          } else if (Qh.prop_grouped == kPropSmall) {
            IFGF_TIMED(7, (prop_small_kernel<PS, PA, T, MAXR, 1, SPLIT>
                           <<<(unsigned)Qh.nschunks, 64, 0, st>>>(A, l, Vcur, Vnext)));
            done = true;
          } else if (Qh.prop_grouped == kPropMedium) {
            IFGF_TIMED(7, (prop_small_kernel<PS, PA, T, MAXR, kMediumWaves, SPLIT>
                           <<<(unsigned)Qh.nmchunks, 64 * kMediumWaves, 0, st>>>(A, l, Vcur,
                                                                                 Vnext)));
            done = true;
          } else if (Qh.prop_grouped == kPropLean) {
            IFGF_TIMED(7, (prop_small_kernel<PS, PA, T, MAXR, kMediumWaves, SPLIT, kLeanBoxes>
                           <<<(unsigned)Qh.nlchunks, 64 * kMediumWaves, 0, st>>>(A, l, Vcur,
                                                                                 Vnext)));
            done = true;
          }
        }
        if (!done)
          IFGF_TIMED(4, (launch_prop_node<PS, PA, T, MAXR>(A, l, Vcur, Vnext, Qh.ncones, st)));
        CT* tmp = Vcur;
        Vcur = Vnext;
        Vnext = tmp;
      }
    }
  }
  IFGF_TIMED(5, (perm_out_kernel<T><<<nblk(nr, 256), 256, 0, st>>>(
                    os, (CT*)out_user, A.perm, A.n, A.nrhs)));
  return hipGetLastError();
}

template <int PS, int PA, typename T, int MAXR, bool SPLIT>
static hipError_t prop_level_impl(const ApplyArgs& A, int l, int kind,
                                  hipStream_t st) {
  typedef typename C2<T>::type CT;
  constexpr int P = PS * PA * PA;
  const StepDev& Qh = A.step_host[l + 1];
  CT* Vc = (CT*)A.vbuf[0];
  CT* Vp = (CT*)A.vbuf[1];
  if (Qh.ncones <= 0) return hipSuccess;
  if constexpr (P <= kMfmaMaxP) {
    if (kind == kPropGrouped && Qh.nchunks > 0) {
      launch_grouped<PS, PA, T, MAXR>(A, l, Vc, Vp, Qh.nchunks, st);
      return hipGetLastError();
    }
    if (kind == kPropSmall && Qh.nschunks > 0) {
      prop_small_kernel<PS, PA, T, MAXR, 1, SPLIT><<<(unsigned)Qh.nschunks, 64, 0, st>>>(A, l, Vc, Vp);
      return hipGetLastError();
    }
    if (kind == kPropLean && Qh.nlchunks > 0) {
      prop_small_kernel<PS, PA, T, MAXR, kMediumWaves, SPLIT, kLeanBoxes>
          <<<(unsigned)Qh.nlchunks, 64 * kMediumWaves, 0, st>>>(A, l, Vc, Vp);
      return hipGetLastError();
    }
    if (kind == kPropMedium && Qh.nmchunks > 0) {
      prop_small_kernel<PS, PA, T, MAXR, kMediumWaves, SPLIT>
          <<<(unsigned)Qh.nmchunks, 64 * kMediumWaves, 0, st>>>(A, l, Vc, Vp);
      return hipGetLastError();
    }
  }
  launch_prop_node<PS, PA, T, MAXR>(A, l, Vc, Vp, Qh.ncones, st);
  return hipGetLastError();
}

int prop_table_record_bytes(int ps, int pa, int precision) {
  const int P = ps * pa * pa;
  if (P == 75) return precision == 0 ? OctRec<75, double>::kSize : OctRec<75, float>::kSize;
  if (P == 18) return precision == 0 ? OctRec<18, double>::kSize : OctRec<18, float>::kSize;
  if (P == 245) return 0;  // no matrix-core propagation at (5, 7)
  return 0;
}

hipError_t launch_prop_table(const ApplyArgs& A, int l, int ps, int pa, int precision,
                             int64_t ngroups, hipStream_t st) {
  if (ngroups <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)(ngroups * 8);
#define IFGF_PT(PS_, PA_)                                                           \
  if (ps == PS_ && pa == PA_) {                                                     \
    if (precision == 0)                                                             \
      prop_table_kernel<PS_, PA_, double><<<blocks, 64, 0, st>>>(A, l);             \
    else                                                                            \
      prop_table_kernel<PS_, PA_, float><<<blocks, 64, 0, st>>>(A, l);              \
    return hipGetLastError();                                                       \
  }
  IFGF_PT(3, 5)
  IFGF_PT(2, 3)
#undef IFGF_PT
  return hipErrorInvalidValue;
}

hipError_t launch_prop_level(const ApplyArgs& A, int l, int ps, int pa,
                             int precision, int kind, hipStream_t st) {
#define IFGF_PL(PS_, PA_)                                                      \
  if (ps == PS_ && pa == PA_) {                                                \
    if (precision == 0)                                                        \
      return A.nrhs <= 1 ? prop_level_impl<PS_, PA_, double, 1, false>(A, l, kind, st) \
                         : prop_level_impl<PS_, PA_, double, kMaxRhs, false>(A, l, kind, st); \
    if (precision == 2)                                                        \
      return A.nrhs <= 1 ? prop_level_impl<PS_, PA_, float, 1, true>(A, l, kind, st) \
                         : prop_level_impl<PS_, PA_, float, kMaxRhs, true>(A, l, kind, st); \
    return A.nrhs <= 1 ? prop_level_impl<PS_, PA_, float, 1, false>(A, l, kind, st) \
                       : prop_level_impl<PS_, PA_, float, kMaxRhs, false>(A, l, kind, st); \
  }
  IFGF_PL(3, 5)
  IFGF_PL(2, 3)
  IFGF_PL(5, 7)
#undef IFGF_PL
  return hipErrorInvalidValue;
}

// Workspace of the allocation-free apply: one static device array per GPU,
// held from the first use of the library on that GPU until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in); it passes the device address that
// hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_apply(const ApplyArgs& A, int ps, int pa, int precision,
                        const void* dens_user, void* out_user, hipStream_t st,
                        Profiler* prof) {
#define IFGF_APPLY(PS_, PA_)                                                  \
  if (ps == PS_ && pa == PA_) {                                               \
    if (precision == 0)                                                       \
      return A.nrhs <= 1                                                      \
                 ? apply_impl<PS_, PA_, double, 1, false>(A, dens_user, out_user, st, prof) \
                 : apply_impl<PS_, PA_, double, kMaxRhs, false>(A, dens_user, out_user, st, prof); \
    if (precision == 2)                                                       \
      return A.nrhs <= 1                                                      \
                 ? apply_impl<PS_, PA_, float, 1, true>(A, dens_user, out_user, st, prof) \
                 : apply_impl<PS_, PA_, float, kMaxRhs, true>(A, dens_user, out_user, st, prof); \
    return A.nrhs <= 1                                                        \
               ? apply_impl<PS_, PA_, float, 1, false>(A, dens_user, out_user, st, prof) \
               : apply_impl<PS_, PA_, float, kMaxRhs, false>(A, dens_user, out_user, st, prof); \
  }
  IFGF_APPLY(3, 5)
  IFGF_APPLY(2, 3)
  IFGF_APPLY(5, 7)
#undef IFGF_APPLY
  return hipErrorInvalidValue;
}

}  // namespace ifgf
