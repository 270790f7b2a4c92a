// ifgf_api.cpp -- the C ABI of libifgf.so (declared in include/ifgf.h).
//
// Plan construction: host octree and interaction lists (host_tree.cpp),
// upload, then the relevant cone segments of eq. (relevantconesegments)
// built on the GPU top-down (level 3 first, i.e. the highest step first):
// a cone of box k is relevant if it holds a cousin point of k or a node of
// a relevant cone of k's parent.  Apply: permute in, near field, leaf
// evaluations, then per level interpolation and propagation, permute out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ifgf.h"
#include "host_tree.h"
#include "ifgf_device.h"

using namespace ifgf;

namespace {

thread_local std::string g_err;

const double kPi = 3.14159265358979323846;

ifgf_status fail(ifgf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIP_TRY(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) throw HipError{e_, #call};    \
  } while (0)

}  // namespace

struct ifgf_plan_s {
  int p_s = 0, p_ang = 0;
  ifgf_opts opts{};
  bool grid_doubling = true;  // the cone grid doubles per level up
  std::string tune_cache;     // copy of opts.tune_cache
  Merged m;
  ifgf_info info{};
  // Device state.
  int device = -1;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  int64_t bytes = 0;
  ApplyArgs A{};
  int64_t ws_vbytes = 0;      // bytes of one cone-value buffer (vbuf[0], vbuf[1])
  int64_t ws_pbytes = 0;      // bytes of the sorted densities (and of the sorted output)
  std::vector<StepDev> steps_h;
  StepDev* steps_d = nullptr;
  bool device_ready = false;
  // Profiling.
  bool profiling = false;
  std::vector<Profiler::Rec> prof_recs;
  int prof_pending = 0;
  double prof_ms[IFGF_N_STAGES] = {0};
  int64_t prof_launches[IFGF_N_STAGES] = {0};
  // Captured apply.
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* g_dens = nullptr;
  void* g_out = nullptr;

  template <class T>
  T* dalloc(int64_t count) {
    if (count <= 0) count = 1;
    void* p = nullptr;
    size_t nbytes = sizeof(T) * (size_t)count;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) throw HipError{e, "hipMalloc"};
    allocs.push_back(p);
    bytes += (int64_t)nbytes;
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>((int64_t)v.size());
    if (!v.empty())
      HIP_TRY(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return p;
  }
  void dfree(void* p) {
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) allocs.erase(it);
    (void)hipFree(p);
  }
  ~ifgf_plan_s() {
    for (void* p : allocs) (void)hipFree(p);
    for (auto& r : prof_recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

static ifgf_status validate(int p_s, int p_ang, const ifgf_opts& o) {
  if (p_s < 1 || p_ang < 1) return fail(IFGF_EINVAL, "p_s and p_ang must be >= 1");
  if (o.precision != IFGF_FP64 && o.precision != IFGF_FP32_MIXED &&
      o.precision != IFGF_FP32_BF16X3)
    return fail(IFGF_EINVAL, "unknown precision");
  if (o.n_rhs < 1) return fail(IFGF_EINVAL, "n_rhs must be >= 1");
  if (o.n_rhs > kMaxRhs) return fail(IFGF_EUNSUPPORTED, "n_rhs > 4 is not supported");
  for (int a = 0; a < 3; ++a)
    if (o.leaf_grid[a] < 1 || o.leaf_grid[a] > 4096)
      return fail(IFGF_EINVAL, "leaf_grid entries must be in [1, 4096]");
  if (o.levels != 0 && o.levels < 3) return fail(IFGF_EINVAL, "levels must be 0 or >= 3");
  if (o.stages < 0 || o.stages > 3) return fail(IFGF_EINVAL, "stages must be in [0, 3]");
  if (o.prop_kernel < 0 || o.prop_kernel > 5) return fail(IFGF_EINVAL, "prop_kernel must be 0..5");
  if (o.lookup < 0 || o.lookup > 1) return fail(IFGF_EINVAL, "lookup must be 0 or 1");
  if (!(o.cone_margin >= 0.0 && o.cone_margin < 0.25))
    return fail(IFGF_EINVAL, "cone_margin must be in [0, 0.25)");
  if (o.grid_rule < 0 || o.grid_rule > 2) return fail(IFGF_EINVAL, "grid_rule must be 0, 1 or 2");
  if (o.prop_tables < 0 || o.prop_tables > 2) return fail(IFGF_EINVAL, "prop_tables must be 0, 1 or 2");
  bool ok = (p_s == 3 && p_ang == 5) || (p_s == 2 && p_ang == 3) || (p_s == 5 && p_ang == 7);
  if (!ok && !o.host_only)
    return fail(IFGF_EUNSUPPORTED, "no kernel compiled for this (p_s, p_ang)");
  return IFGF_OK;
}

static uint64_t next_pow2(uint64_t v) {
  uint64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

static int bits_for(uint64_t v) {
  int b = 1;
  while (b < 64 && (uint64_t(1) << b) <= v) ++b;
  return b;
}

// Chebyshev first-kind nodes and Lagrange product weights.
static void cheb_nodes(int n, double* t, double* w) {
  for (int j = 0; j < n; ++j) t[j] = std::cos((2.0 * j + 1.0) * kPi / (2.0 * n));
  for (int j = 0; j < n; ++j) {
    double p = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) p *= (t[j] - t[m]);
    w[j] = 1.0 / p;
  }
}

#ifndef IFGF_BUILD_ID
#define IFGF_BUILD_ID "unversioned"
#endif

// Key of a plan in the tuning cache: the library build (a hash of its
// sources), the GPU architecture, precision, RHS count, interpolation order
// and a hash of the plan's shape (points, instances, and per step the
// boxes, relevant cones, grid and propagation chunk counts).
static std::string tune_key(ifgf_plan_s* P) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a, 64 bit
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)P->m.n);
  mix((uint64_t)P->m.n_inst);
  mix((uint64_t)P->A.n_steps);
  for (const StepDev& S : P->steps_h) {
    mix((uint64_t)S.nb);
    mix((uint64_t)S.ncones);
    mix((uint64_t)S.ngrid);
    mix((uint64_t)S.nchunks);
    mix((uint64_t)S.nschunks);
    mix((uint64_t)S.nmchunks);
    mix((uint64_t)S.nlchunks);
  }
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, P->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == '|') c = '_';
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s %s prec=%d rhs=%d p=%d,%d shape=%016llx", IFGF_BUILD_ID,
                arch.c_str(), P->opts.precision, P->opts.n_rhs, P->p_s, P->p_ang,
                (unsigned long long)h);
  return buf;
}

// Kernels recorded for this plan's key in the tuning cache file, one per
// step ("-" where not tuned); false when the file has no such line.
static bool tune_cache_read(const std::string& path, const std::string& key,
                            std::vector<int>& modes) {
  std::FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (!found && std::fgets(line, sizeof(line), f)) {
    std::string ln(line);
    size_t bar = ln.find(" | modes=");
    if (bar == std::string::npos || ln.compare(0, bar, key) != 0 || bar != key.size()) continue;
    std::vector<int> got;
    const char* p = ln.c_str() + bar + 9;
    while (*p && *p != '\n' && *p != ' ') {
      if (*p == '-') {
        got.push_back(-1);
        ++p;
      } else {
        char* e = nullptr;
        long v = std::strtol(p, &e, 10);
        if (e == p) break;
        got.push_back((int)v);
        p = e;
      }
      if (*p == ',') ++p;
    }
    if (got.size() == modes.size()) {
      modes = got;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void tune_cache_append(const std::string& path, const std::string& key,
                              const std::vector<int>& modes) {
  std::FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;  // an unwritable cache only costs the next plan a re-tune
  std::string ln = key + " | modes=";
  for (size_t i = 0; i < modes.size(); ++i) {
    if (i) ln += ",";
    ln += modes[i] < 0 ? std::string("-") : std::to_string(modes[i]);
  }
  ln += "\n";
  std::fputs(ln.c_str(), f);
  std::fclose(f);
}

// Time the four propagation kernels on every level where the matrix-core
// forms apply (zeroed cone values: the kernels' work does not depend on the
// values) and keep the fastest.  With a tuning cache, a recorded choice for
// the same key is taken without timing.
static void autotune(ifgf_plan_s* P) {
  ApplyArgs& A = P->A;
  hipStream_t st = P->stream;
  const int PP = P->p_s * P->p_ang * P->p_ang;
  if (PP > kMfmaMaxP) return;
  std::string key;
  if (!P->tune_cache.empty()) {
    key = tune_key(P);
    std::vector<int> modes(A.n_steps, -1);
    if (tune_cache_read(P->tune_cache, key, modes)) {
      for (int l = 1; l < A.n_steps; ++l) {
        StepDev& Q = P->steps_h[l];
        if (modes[l] >= kPropNode && modes[l] < kPropKinds && Q.ncones > 0 && Q.nchunks > 0)
          Q.prop_grouped = modes[l];
      }
      P->info.tune_cache_hit = 1;
      HIP_TRY(hipMemcpy(P->steps_d, P->steps_h.data(), sizeof(StepDev) * A.n_steps,
                        hipMemcpyHostToDevice));
      return;
    }
  }
  size_t csize = P->opts.precision == IFGF_FP64 ? 16 : 8;
  int64_t maxc = 1;
  for (int l = 0; l < A.n_steps; ++l) maxc = std::max<int64_t>(maxc, P->steps_h[l].ncones);
  HIP_TRY(hipMemsetAsync(A.vbuf[0], 0, maxc * A.nrhs * PP * csize, st));
  HIP_TRY(hipMemsetAsync(A.vbuf[1], 0, maxc * A.nrhs * PP * csize, st));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  for (int l = 0; l + 1 < A.n_steps; ++l) {
    StepDev& Q = P->steps_h[l + 1];
    if (Q.ncones == 0 || Q.nchunks == 0) continue;
    // Each form: a timed warm-up launch, then two timed launches, unless the
    // warm-up alone is 1.5 times the best so far (then it stands for the form;
    // the slow forms of a level cost one launch).  The rule-based choice goes
    // first, so that the others are measured against a good form.
    float best[kPropKinds] = {0, 0, 0, 0, 0};
    int pick = -1;
    for (int q = 0; q < kPropKinds; ++q) {
      const int g = q == 0 ? Q.prop_grouped : (q <= Q.prop_grouped ? q - 1 : q);
      float warm = 0;
      HIP_TRY(hipEventRecord(e0, st));
      HIP_TRY(launch_prop_level(A, l, P->p_s, P->p_ang, P->opts.precision, g, st));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&warm, e0, e1));
      if (pick >= 0 && warm > 1.5f * best[pick] / 2) {
        best[g] = 2 * warm;
        continue;
      }
      HIP_TRY(hipEventRecord(e0, st));
      for (int rep = 0; rep < 2; ++rep)
        HIP_TRY(launch_prop_level(A, l, P->p_s, P->p_ang, P->opts.precision, g, st));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&best[g], e0, e1));
      if (pick < 0 || best[g] < best[pick]) pick = g;
    }
    Q.prop_grouped = pick;
    for (int g = 0; g < kPropKinds; ++g) P->info.autotune_ms[l + 1][g] = best[g] / 2;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!P->tune_cache.empty()) {
    std::vector<int> modes(A.n_steps, -1);
    for (int l = 1; l < A.n_steps; ++l) {
      const StepDev& Q = P->steps_h[l];
      if (Q.ncones > 0 && Q.nchunks > 0) modes[l] = Q.prop_grouped;
    }
    tune_cache_append(P->tune_cache, key, modes);
  }
  HIP_TRY(hipMemcpy(P->steps_d, P->steps_h.data(), sizeof(StepDev) * A.n_steps,
                    hipMemcpyHostToDevice));
}

// Plan-time tables of the matrix-core propagation: the box-independent
// record (node geometry seen from each child octant, grouping of the nodes
// by child cone) of every (instance, gamma') group of a step, so that the
// apply reads it instead of recomputing it for every chunk of boxes.
// Steps are taken from the leaf upwards (where groups hold the most boxes)
// while the tables stay within the budget: four times the bytes of one
// cone-value buffer (at least 1 GiB) with prop_tables = 0, none with 1, all
// with 2.
static void build_prop_tables(ifgf_plan_s* P, int64_t vbytes) {
  ApplyArgs& A = P->A;
  const int rec = prop_table_record_bytes(P->p_s, P->p_ang, P->opts.precision);
  if (rec <= 0 || P->opts.prop_tables == 1) return;
  int64_t budget = P->opts.prop_tables == 2 ? INT64_MAX
                                             : std::max<int64_t>(4 * vbytes, int64_t(1) << 30);
  // The tables only save work: they never take the device's last memory (a
  // tenth of it, at least 4 GiB, stays free for the caller).
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  const int64_t reserve = std::max<int64_t>((int64_t)(total_b / 10), int64_t(4) << 30);
  budget = std::min<int64_t>(budget, std::max<int64_t>(0, (int64_t)free_b - reserve));
  int64_t used = 0;
  for (int l = 1; l < A.n_steps; ++l) {
    StepDev& Q = P->steps_h[l];
    if (Q.ngroups <= 0 || Q.ncones <= 0) continue;
    const int64_t bytes = Q.ngroups * 8 * (int64_t)rec;
    if (used + bytes > budget) break;
    Q.prop_table = P->dalloc<unsigned char>(bytes);
    used += bytes;
    HIP_TRY(hipMemcpy(P->steps_d, P->steps_h.data(), sizeof(StepDev) * A.n_steps,
                      hipMemcpyHostToDevice));
    HIP_TRY(launch_prop_table(A, l - 1, P->p_s, P->p_ang, P->opts.precision, Q.ngroups,
                              P->stream));
  }
  P->info.prop_table_bytes = used;
}

static void build_device(ifgf_plan_s* P) {
  Merged& m = P->m;
  const int ps = P->p_s, pa = P->p_ang, PP = ps * pa * pa;
  const int L = m.n_steps;
  hipStream_t st = P->stream;
  ApplyArgs& A = P->A;
  A.n = m.n;
  A.nrhs = P->opts.n_rhs;
  A.n_steps = L;
  A.stages = P->opts.stages == 0 ? 3 : P->opts.stages;
  A.x = P->upload(m.xs[0]);
  A.y = P->upload(m.xs[1]);
  A.z = P->upload(m.xs[2]);
  A.perm = P->upload(m.perm);
  // Leaf-box-relative FP32 source offsets for LevelDEvaluations.
  A.q_leaf = nullptr;
  if (P->opts.precision != IFGF_FP64 && L > 0) {
    const MergedStep& S0 = m.step[0];
    std::vector<float4> q((size_t)m.n, float4{0.f, 0.f, 0.f, 0.f});
    for (int64_t b = 0; b < S0.nb; ++b)
      for (int64_t i = S0.first[b]; i < (int64_t)S0.first[b] + S0.count[b]; ++i) {
        const float q0 = (float)(m.xs[0][i] - S0.center[3 * b]);
        const float q1 = (float)(m.xs[1][i] - S0.center[3 * b + 1]);
        const float q2 = (float)(m.xs[2][i] - S0.center[3 * b + 2]);
        q[i] = float4{q0, q1, q2, q0 * q0 + q1 * q1 + q2 * q2};
      }
    A.q_leaf = P->upload(q);
  }
  A.inst_kappa = P->upload(m.inst_kappa);
  A.nbr_begin = P->upload(m.nbr_begin);
  A.nbr = P->upload(m.nbr);
  std::memset(&A.cheb, 0, sizeof(A.cheb));
  cheb_nodes(ps, A.cheb.ts, A.cheb.ws);
  cheb_nodes(pa, A.cheb.ta, A.cheb.wa);
  A.err = P->dalloc<int>(1);
  HIP_TRY(hipMemset(A.err, 0, sizeof(int)));

  const double eta = std::sqrt(3.0) / 3.0;
  P->steps_h.assign(L, StepDev{});
  for (int l = 0; l < L; ++l) {
    MergedStep& S = m.step[l];
    StepDev& D = P->steps_h[l];
    D.nb = S.nb;
    D.center = P->upload(S.center);
    D.inst = P->upload(S.inst);
    D.first = P->upload(S.first);
    D.count = P->upload(S.count);
    D.child = l >= 1 ? P->upload(S.child) : nullptr;
    D.cous_begin = P->upload(S.cous_begin);
    D.cous = P->upload(S.cous);
    D.pt_box = P->upload(S.pt_box);
    D.inst_h = P->upload(S.inst_h);
    D.inst_H = P->upload(S.inst_H);
    // Cone grid: the leaf grid, doubled per dimension for every level up
    // when it follows the wavelength (grid_rule).
    const int gs = P->grid_doubling ? l : 0;
    D.ns = P->opts.leaf_grid[0] << gs;
    D.nt = P->opts.leaf_grid[1] << gs;
    D.np = P->opts.leaf_grid[2] << gs;
    D.ngrid = (int64_t)D.ns * D.nt * D.np;
    D.ds = eta / D.ns;
    D.dt = kPi / D.nt;
    D.dp = 2.0 * kPi / D.np;
    std::vector<double> sn((size_t)D.ns * ps), tn((size_t)D.nt * pa * 2), pn((size_t)D.np * pa * 2);
    for (int i = 0; i < D.ns; ++i)
      for (int a = 0; a < ps; ++a)
        sn[(size_t)i * ps + a] = D.ds * (double(i) + 0.5 * (A.cheb.ts[a] + 1.0));
    for (int i = 0; i < D.nt; ++i)
      for (int b = 0; b < pa; ++b) {
        double th = D.dt * (double(i) + 0.5 * (A.cheb.ta[b] + 1.0));
        tn[2 * ((size_t)i * pa + b)] = std::sin(th);
        tn[2 * ((size_t)i * pa + b) + 1] = std::cos(th);
      }
    for (int i = 0; i < D.np; ++i)
      for (int c = 0; c < pa; ++c) {
        double ph = D.dp * (double(i) + 0.5 * (A.cheb.ta[c] + 1.0));
        pn[2 * ((size_t)i * pa + c)] = std::sin(ph);
        pn[2 * ((size_t)i * pa + c) + 1] = std::cos(ph);
      }
    D.s_node = P->upload(sn);
    D.t_node = P->upload(tn);
    D.p_node = P->upload(pn);
    D.rds = 1.0 / D.ds;
    D.rdt = 1.0 / D.dt;
    D.rdp = 1.0 / D.dp;
    std::vector<double> tb((size_t)(D.nt + 1) * 2), pb((size_t)(D.np + 1) * 2);
    for (int i = 0; i <= D.nt; ++i) {
      tb[2 * (size_t)i] = std::cos(D.dt * i);
      tb[2 * (size_t)i + 1] = std::sin(D.dt * i);
    }
    for (int i = 0; i <= D.np; ++i) {
      pb[2 * (size_t)i] = std::cos(D.dp * i);
      pb[2 * (size_t)i + 1] = std::sin(D.dp * i);
    }
    D.t_bnd = P->upload(tb);
    D.p_bnd = P->upload(pb);
    D.ncones = 0;
  }
  P->steps_d = P->dalloc<StepDev>(std::max(L, 1));
  A.step = P->steps_d;
  A.step_host = P->steps_h.data();
  auto sync_steps = [&]() {
    HIP_TRY(hipMemcpy(P->steps_d, P->steps_h.data(), sizeof(StepDev) * L,
                      hipMemcpyHostToDevice));
  };
  sync_steps();

  // Relevant cones, top-down.
  unsigned int* counters = P->dalloc<unsigned int>(2);
  int* overflow = P->dalloc<int>(1);
  for (int l = L - 1; l >= 0; --l) {
    StepDev& D = P->steps_h[l];
    // Unique (box, cone) keys are bounded by the grid, and in practice by
    // ~2 per (box, cousin box) pair plus a few per parent cone.
    int64_t pairs = (int64_t)m.step[l].cous.size();
    uint64_t est = (uint64_t)std::min<double>(
        (double)D.nb * (double)D.ngrid,
        2.0 * (double)pairs +
            (l + 1 < L ? (double)P->steps_h[l + 1].ncones * 8.0 : 0.0) + 4096.0);
    uint64_t cap = next_pow2(std::max<uint64_t>(4096, 2 * est));
    unsigned long long* tab = nullptr;
    unsigned int count = 0;
    for (int attempt = 0;; ++attempt) {
      tab = P->dalloc<unsigned long long>((int64_t)cap);
      HIP_TRY(launch_fill_u64(tab, (int64_t)cap, kEmptyKey, st));
      HIP_TRY(hipMemsetAsync(counters, 0, 2 * sizeof(unsigned int), st));
      HIP_TRY(hipMemsetAsync(overflow, 0, sizeof(int), st));
      MarkArgs M{tab, (unsigned long long)(cap - 1), counters, overflow, P->opts.cone_margin};
      HIP_TRY(launch_mark(A, l, ps, pa, M, st));
      int ovf = 0;
      HIP_TRY(hipMemcpyAsync(&count, counters, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (!ovf && (double)count <= 0.75 * (double)cap) break;
      P->dfree(tab);
      cap *= 4;
      if (attempt > 8) throw HipError{hipErrorOutOfMemory, "relevant-cone table"};
    }
    // Sorted keys -> slots; final lookup table at <= 50% load.
    unsigned long long* keys = P->dalloc<unsigned long long>(count);
    unsigned long long* tmp = P->dalloc<unsigned long long>(count);
    HIP_TRY(hipMemsetAsync(counters + 1, 0, sizeof(unsigned int), st));
    HIP_TRY(launch_compact(tab, (int64_t)cap, keys, counters + 1, st));
    P->dfree(tab);
    if (count > 0) {
      size_t sbytes = 0;
      int end_bit = bits_for((uint64_t)D.nb * (uint64_t)D.ngrid);
      HIP_TRY(sort_keys(keys, tmp, count, end_bit, nullptr, &sbytes, st));
      void* scratch = P->dalloc<char>((int64_t)sbytes + 16);
      HIP_TRY(sort_keys(keys, tmp, count, end_bit, scratch, &sbytes, st));
      HIP_TRY(hipStreamSynchronize(st));
      P->dfree(scratch);
    }
    P->dfree(tmp);
    uint64_t cap2 = next_pow2(std::max<uint64_t>(1024, 2 * (uint64_t)count));
    unsigned long long* hk = P->dalloc<unsigned long long>((int64_t)cap2);
    int* hv = P->dalloc<int>((int64_t)cap2);
    HIP_TRY(launch_fill_u64(hk, (int64_t)cap2, kEmptyKey, st));
    HIP_TRY(hipMemsetAsync(overflow, 0, sizeof(int), st));
    HIP_TRY(launch_build_lookup(keys, count, hk, hv, cap2 - 1, overflow, st));
    int ovf = 0;
    HIP_TRY(hipMemcpyAsync(&ovf, overflow, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ovf) throw HipError{hipErrorUnknown, "cone lookup table overflow"};
    // Dense look-up table where it is small enough.
    D.table = nullptr;
    if (P->opts.lookup == 0 && (double)D.nb * (double)D.ngrid <= (double)(int64_t(1) << 28)) {
      int* tbl = P->dalloc<int>(D.nb * D.ngrid);
      HIP_TRY(launch_fill_i32(tbl, D.nb * D.ngrid, -1, st));
      HIP_TRY(launch_scatter_table(keys, count, tbl, st));
      D.table = tbl;
    }
    // Work counts of this step (for throughput and roofline figures), and
    // the grouping of its cones by (instance, gamma) for propagation.
    {
      std::vector<unsigned long long> hkeys(count);
      if (count > 0)
        HIP_TRY(hipMemcpy(hkeys.data(), keys, sizeof(unsigned long long) * count,
                          hipMemcpyDeviceToHost));
      const MergedStep& S = m.step[l];
      D.prop_grouped = kPropNode;
      D.nchunks = 0;
      D.nschunks = 0;
      D.nmchunks = 0;
      D.nlchunks = 0;
      D.ngroups = 0;
      D.prop_table = nullptr;
      if (l >= 1 && count > 0) {
        const uint64_t ng = (uint64_t)D.ngrid;
        // Slots sorted by (instance, gamma, slot): the composite key
        // instance * grid + gamma of every cone, radix-sorted on the device
        // with the slot as value (stable, so equal keys stay in slot order;
        // a host sort was most of the plan time at a million points).
        std::vector<uint64_t> gkey((size_t)count);
        std::vector<int32_t> order((size_t)count);
        {
          unsigned long long* gk = P->dalloc<unsigned long long>((int64_t)count);
          unsigned long long* gk2 = P->dalloc<unsigned long long>((int64_t)count);
          int* ix = P->dalloc<int>((int64_t)count);
          int* ix2 = P->dalloc<int>((int64_t)count);
          HIP_TRY(launch_group_keys(keys, (int64_t)count, ng, D.inst, gk, ix, st));
          const int gbits = bits_for((uint64_t)m.n_inst * ng);
          size_t sbytes = 0;
          HIP_TRY(sort_pairs(gk, gk2, ix, ix2, (int64_t)count, gbits, nullptr, &sbytes, st));
          void* scratch = P->dalloc<char>((int64_t)sbytes + 16);
          HIP_TRY(sort_pairs(gk, gk2, ix, ix2, (int64_t)count, gbits, scratch, &sbytes, st));
          HIP_TRY(hipMemcpyAsync(gkey.data(), gk2, sizeof(uint64_t) * count,
                                 hipMemcpyDeviceToHost, st));
          HIP_TRY(hipMemcpyAsync(order.data(), ix2, sizeof(int32_t) * count,
                                 hipMemcpyDeviceToHost, st));
          HIP_TRY(hipStreamSynchronize(st));
          P->dfree(scratch);
          P->dfree(ix2);
          P->dfree(ix);
          P->dfree(gk2);
          P->dfree(gk);
        }
        // Chunks of at most cbox (block kernel) and sbox (one-wave kernel)
        // boxes sharing (instance, gamma).
        const int cbox = chunk_boxes(P->opts.precision, P->opts.n_rhs);
        const int sbox = small_chunk_boxes(P->opts.n_rhs, 1);
        const int mbox = small_chunk_boxes(P->opts.n_rhs, kMediumWaves);
        const int lbox = small_chunk_boxes(P->opts.n_rhs, kMediumWaves, kLeanBoxes);
        std::vector<int64_t> cstart, sstart, mstart, lstart, gfirst;
        std::vector<int32_t> clen, slen, mlen, llen, sgroup, mgroup, lgroup;
        int64_t groups = 0;
        for (int64_t i = 0; i < (int64_t)count; ++i) {
          bool same = i > 0 && gkey[i] == gkey[i - 1];
          if (!same) {
            ++groups;
            gfirst.push_back(i);
          }
          if (!same || clen.back() == cbox) {
            cstart.push_back(i);
            clen.push_back(0);
          }
          clen.back() += 1;
          if (!same || slen.back() == sbox) {
            sstart.push_back(i);
            slen.push_back(0);
            sgroup.push_back((int32_t)(groups - 1));
          }
          slen.back() += 1;
          if (!same || mlen.back() == mbox) {
            mstart.push_back(i);
            mlen.push_back(0);
            mgroup.push_back((int32_t)(groups - 1));
          }
          mlen.back() += 1;
          if (!same || llen.back() == lbox) {
            lstart.push_back(i);
            llen.push_back(0);
            lgroup.push_back((int32_t)(groups - 1));
          }
          llen.back() += 1;
        }
        // Without the autotuner: the four-wave task kernel where many boxes
        // share a parent cone index (>= 32 on average), the one-wave task
        // kernel where a few do (>= 4), the per-node kernel otherwise; the
        // block kernel only when asked for.
        double mean = (double)count / (double)std::max<int64_t>(groups, 1);
        int mode = P->opts.prop_kernel;
        if (PP <= kMfmaMaxP) {
          if (mode == 2)
            D.prop_grouped = kPropGrouped;
          else if (mode == 5)
            D.prop_grouped = kPropLean;
          else if (mode == 4 || (mode == 0 && mean >= 32.0))
            D.prop_grouped = kPropMedium;
          else if (mode == 3 || (mode == 0 && mean >= 4.0))
            D.prop_grouped = kPropSmall;
        }
        if (PP <= kMfmaMaxP && (D.prop_grouped != kPropNode || P->opts.autotune)) {
          D.gslot = P->upload(order);
          D.chunk_start = P->upload(cstart);
          D.chunk_len = P->upload(clen);
          D.nchunks = (int64_t)cstart.size();
          // Dispatch order of the task chunks: by the first box of the chunk
          // in buckets of 64 boxes (Morton order), then by group.  Chunks
          // working on nearby boxes for different parent cone indices, which
          // read the same child cones, then run at about the same time and
          // find more of them in the cache (4-5% faster than group order at
          // the dense steps of the 321k-point sphere).
          auto box_order = [&](std::vector<int64_t>& st, std::vector<int32_t>& ln,
                               std::vector<int32_t>& gr) {
            const size_t nc = st.size();
            std::vector<int64_t> bucket(nc);
            for (size_t c = 0; c < nc; ++c)
              bucket[c] = (int64_t)(hkeys[order[st[c]]] / ng) / 64;
            std::vector<size_t> idx(nc);
            for (size_t c = 0; c < nc; ++c) idx[c] = c;
            std::stable_sort(idx.begin(), idx.end(),
                             [&](size_t x, size_t y) { return bucket[x] < bucket[y]; });
            std::vector<int64_t> st2(nc);
            std::vector<int32_t> ln2(nc), gr2(nc);
            for (size_t c = 0; c < nc; ++c) {
              st2[c] = st[idx[c]];
              ln2[c] = ln[idx[c]];
              gr2[c] = gr[idx[c]];
            }
            st.swap(st2);
            ln.swap(ln2);
            gr.swap(gr2);
          };
          box_order(sstart, slen, sgroup);
          box_order(mstart, mlen, mgroup);
          box_order(lstart, llen, lgroup);
          D.schunk_start = P->upload(sstart);
          D.schunk_len = P->upload(slen);
          D.nschunks = (int64_t)sstart.size();
          D.mchunk_start = P->upload(mstart);
          D.mchunk_len = P->upload(mlen);
          D.nmchunks = (int64_t)mstart.size();
          D.ngroups = groups;
          D.group_first = P->upload(gfirst);
          D.schunk_group = P->upload(sgroup);
          D.mchunk_group = P->upload(mgroup);
          D.lchunk_start = P->upload(lstart);
          D.lchunk_len = P->upload(llen);
          D.nlchunks = (int64_t)lstart.size();
          D.lchunk_group = P->upload(lgroup);
        }
      }
      int64_t pairs_l = 0;
      for (unsigned long long k : hkeys) {
        int64_t b = (int64_t)(k / (unsigned long long)D.ngrid);
        if (l == 0) {
          pairs_l += (int64_t)PP * S.count[b];
        } else {
          int nch = 0;
          for (int o = 0; o < 8; ++o) nch += S.child[8 * b + o] >= 0;
          pairs_l += (int64_t)PP * nch;
        }
      }
      if (l == 0) P->info.leaf_pairs = pairs_l;
      else P->info.prop_pairs[l] = pairs_l;
    }
    D.ncones = count;
    D.cone_key = keys;
    D.hkey = hk;
    D.hval = hv;
    D.hmask = cap2 - 1;
    sync_steps();
  }

  // Value buffers (two consecutive levels), sorted densities and output.
  size_t csize = P->opts.precision == IFGF_FP64 ? 16 : 8;
  int64_t maxc = 1;
  for (int l = 0; l < L; ++l) maxc = std::max<int64_t>(maxc, P->steps_h[l].ncones);
  int64_t vbytes = maxc * A.nrhs * PP * (int64_t)csize;
  P->ws_vbytes = vbytes;
  P->ws_pbytes = m.n * A.nrhs * (int64_t)csize;
  A.vbuf[0] = P->dalloc<char>(vbytes);
  A.vbuf[1] = P->dalloc<char>(vbytes);
  A.dens_sorted = P->dalloc<char>(m.n * A.nrhs * (int64_t)csize);
  A.out_sorted = P->dalloc<char>(m.n * A.nrhs * (int64_t)csize);
  build_prop_tables(P, vbytes);
  HIP_TRY(hipStreamSynchronize(st));
  if (P->opts.autotune) autotune(P);
  P->device_ready = true;
}

static void fill_info(ifgf_plan_s* P) {
  ifgf_info& I = P->info;
  Merged& m = P->m;
  I.n_points = m.n;
  I.n_instances = m.n_inst;
  I.max_levels = m.max_D;
  I.n_steps = m.n_steps;
  I.p_s = P->p_s;
  I.p_ang = P->p_ang;
  I.n_rhs = P->opts.n_rhs;
  I.precision = P->opts.precision;
  for (int l = 0; l < m.n_steps && l < IFGF_MAX_LEVELS; ++l) {
    I.boxes[l] = m.step[l].nb;
    I.cones[l] = P->device_ready ? P->steps_h[l].ncones : 0;
    int64_t pairs = 0;
    for (int64_t b = 0; b < m.step[l].nb; ++b)
      pairs += (m.step[l].cous_begin[b + 1] - m.step[l].cous_begin[b]) * (int64_t)m.step[l].count[b];
    I.cousin_pairs[l] = pairs;
    const int gs = P->grid_doubling ? l : 0;
    I.grid[l] = (int64_t)(P->opts.leaf_grid[0] << gs) * (P->opts.leaf_grid[1] << gs) *
                (P->opts.leaf_grid[2] << gs);
    I.prop_mode[l] = (l >= 1 && P->device_ready) ? P->steps_h[l].prop_grouped + 1 : 0;
  }
  I.near_pairs = m.near_pairs;
  I.device_bytes = P->bytes;
  I.grid_doubling = P->grid_doubling ? 1 : 0;
}

static ifgf_status plan_common(ifgf_plan_t* out, int n_inst,
                               const int64_t* offsets, const double* points,
                               const double* kappas, int p_s, int p_ang,
                               double leaf_size, const ifgf_opts* opts_in) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out || !points || !kappas || !offsets) return fail(IFGF_EINVAL, "null pointer");
  *out = nullptr;
  if (n_inst < 1) return fail(IFGF_EINVAL, "n_inst must be >= 1");
  ifgf_opts o;
  ifgf_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.leaf_grid[0] == 0 && o.leaf_grid[1] == 0 && o.leaf_grid[2] == 0) {
    o.leaf_grid[0] = 2;
    o.leaf_grid[1] = 4;
    o.leaf_grid[2] = 8;
  }
  ifgf_status s = validate(p_s, p_ang, o);
  if (s != IFGF_OK) return s;
  if (offsets[0] != 0) return fail(IFGF_EINVAL, "offsets[0] must be 0");
  for (int i = 0; i < n_inst; ++i)
    if (offsets[i + 1] - offsets[i] < 2) return fail(IFGF_EINVAL, "every instance needs >= 2 points");
  // Cone grid rule: doubling follows the wavelength; kappa = 0 keeps the
  // leaf grid.  Instances of one plan share the grid of every step.
  int n_zero = 0;
  for (int i = 0; i < n_inst; ++i) n_zero += kappas[i] == 0.0;
  if (o.grid_rule == 0 && n_zero > 0 && n_zero < n_inst)
    return fail(IFGF_EINVAL, "grid_rule 0 cannot mix kappa = 0 and kappa > 0 in one plan");
  ifgf_plan_s* P = new (std::nothrow) ifgf_plan_s();
  if (!P) return fail(IFGF_ENOMEM, "out of host memory");
  P->p_s = p_s;
  P->p_ang = p_ang;
  P->opts = o;
  P->grid_doubling = o.grid_rule == 1 || (o.grid_rule == 0 && n_zero == 0);
  if (o.tune_cache) P->tune_cache = o.tune_cache;
  P->opts.tune_cache = nullptr;  // the plan keeps its own copy
  try {
    // Points may be host or device memory; device points are copied to the
    // host, where the octree is built.
    std::vector<double> host_pts;
    if (!o.host_only) {
      hipPointerAttribute_t attr;
      std::memset(&attr, 0, sizeof(attr));
      hipError_t pe = hipPointerGetAttributes(&attr, points);
      if (pe == hipSuccess && attr.type == hipMemoryTypeDevice) {
        host_pts.resize(3 * (size_t)offsets[n_inst]);
        HIP_TRY(hipMemcpy(host_pts.data(), points, sizeof(double) * host_pts.size(),
                          hipMemcpyDeviceToHost));
        points = host_pts.data();
      } else if (pe != hipSuccess) {
        (void)hipGetLastError();  // unregistered host memory: not an error
      }
    }
    LevelRule rule;
    rule.levels = o.levels;
    rule.leaf_size = leaf_size;
    rule.leaf_max = o.leaf_max;
    rule.leaf_abs = o.leaf_abs;
    std::vector<InstanceTree> trees(n_inst);
    int threads = default_threads();
    for (int i = 0; i < n_inst; ++i) {
      std::string msg;
      int rc = build_instance(points + 3 * offsets[i], offsets[i + 1] - offsets[i],
                              kappas[i], rule, trees[i], msg);
      if (rc != IFGF_OK) {
        delete P;
        return fail((ifgf_status)rc, n_inst > 1 ? "instance " + std::to_string(i) + ": " + msg : msg);
      }
      build_lists(trees[i], threads);
    }
    std::string msg;
    int rc = merge_instances(trees, P->m, msg);
    if (rc != IFGF_OK) {
      delete P;
      return fail((ifgf_status)rc, msg);
    }
    if (!o.host_only) {
      if (o.device >= 0) HIP_TRY(hipSetDevice(o.device));
      HIP_TRY(hipGetDevice(&P->device));
      P->stream = (hipStream_t)o.stream;
      build_device(P);
    }
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(IFGF_ENOMEM, "out of host memory");
  } catch (const HipError& e) {
    delete P;
    ifgf_status st = (e.e == hipErrorOutOfMemory) ? IFGF_ENOMEM : IFGF_EHIP;
    return fail(st, std::string(e.what) + ": " + hipGetErrorString(e.e));
  }
  fill_info(P);
  P->info.plan_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = P;
  return IFGF_OK;
}

extern "C" {

ifgf_status ifgf_default_opts(ifgf_opts* o) {
  if (!o) return fail(IFGF_EINVAL, "null opts");
  std::memset(o, 0, sizeof(*o));
  o->precision = IFGF_FP64;
  o->n_rhs = 1;
  o->leaf_grid[0] = 2;
  o->leaf_grid[1] = 4;
  o->leaf_grid[2] = 8;
  o->levels = 0;
  o->stages = 3;
  o->host_only = 0;
  o->device = -1;
  o->stream = nullptr;
  o->cone_margin = 1e-9;
  return IFGF_OK;
}

ifgf_status ifgf_plan(ifgf_plan_t* plan, const double* points, int64_t n,
                      double kappa, int p_s, int p_ang, double leaf_size) {
  return ifgf_plan_ex(plan, points, n, kappa, p_s, p_ang, leaf_size, nullptr);
}

ifgf_status ifgf_plan_ex(ifgf_plan_t* plan, const double* points, int64_t n,
                         double kappa, int p_s, int p_ang, double leaf_size,
                         const ifgf_opts* opts) {
  int64_t off[2] = {0, n};
  return plan_common(plan, 1, off, points, &kappa, p_s, p_ang, leaf_size, opts);
}

ifgf_status ifgf_plan_batched(ifgf_plan_t* plan, int n_inst,
                              const int64_t* offsets, const double* points,
                              const double* kappas, int p_s, int p_ang,
                              double leaf_size, const ifgf_opts* opts) {
  return plan_common(plan, n_inst, offsets, points, kappas, p_s, p_ang,
                     leaf_size, opts);
}

ifgf_status ifgf_apply(ifgf_plan_t P, const void* dens, void* out) {
  if (!P || !dens || !out) return fail(IFGF_EINVAL, "null argument");
  if (!P->device_ready) return fail(IFGF_EINVAL, "plan was built host-only");
  hipError_t e = hipSetDevice(P->device);
  Profiler prof;
  Profiler* pp = nullptr;
  if (e == hipSuccess && P->profiling) {
    // Room for every launch of one apply.
    size_t need = (size_t)P->prof_pending + 8 + 2 * (size_t)P->A.n_steps;
    while (e == hipSuccess && P->prof_recs.size() < need) {
      Profiler::Rec r{0, nullptr, nullptr};
      e = hipEventCreate(&r.a);
      if (e == hipSuccess) e = hipEventCreate(&r.b);
      if (e == hipSuccess) P->prof_recs.push_back(r);
    }
    prof.recs = P->prof_recs.data();
    prof.n = P->prof_pending;
    prof.cap = (int)P->prof_recs.size();
    pp = &prof;
  }
  if (e == hipSuccess)
    e = launch_apply(P->A, P->p_s, P->p_ang, P->opts.precision, dens, out, P->stream, pp);
  if (pp) P->prof_pending = prof.n;
  if (e != hipSuccess)
    return fail(IFGF_EHIP, std::string("apply: ") + hipGetErrorString(e));
  return IFGF_OK;
}

ifgf_status ifgf_apply_graph(ifgf_plan_t P, const void* dens, void* out) {
  if (!P || !dens || !out) return fail(IFGF_EINVAL, "null argument");
  if (!P->device_ready) return fail(IFGF_EINVAL, "plan was built host-only");
  hipError_t e = hipSetDevice(P->device);
  if (e == hipSuccess && (!P->gexec || P->g_dens != dens || P->g_out != out)) {
    if (P->gexec) {
      (void)hipGraphExecDestroy(P->gexec);
      P->gexec = nullptr;
    }
    // Capture on a stream of the library's own; the null stream cannot be
    // captured.  Work already queued on the plan's stream is ordered
    // before the first launch by the launch itself.
    if (!P->cap_stream) e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      hipError_t le = launch_apply(P->A, P->p_s, P->p_ang, P->opts.precision, dens, out,
                                   P->cap_stream, nullptr);
      e = hipStreamEndCapture(P->cap_stream, &graph);
      if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) {
      P->g_dens = dens;
      P->g_out = out;
    } else {
      P->gexec = nullptr;
    }
  }
  if (e == hipSuccess) e = hipGraphLaunch(P->gexec, P->stream);
  if (e != hipSuccess)
    return fail(IFGF_EHIP, std::string("apply_graph: ") + hipGetErrorString(e));
  return IFGF_OK;
}

ifgf_status ifgf_apply_noalloc(ifgf_plan_t P, const void* dens, void* out) {
  if (!P || !dens || !out) return fail(IFGF_EINVAL, "null argument");
  if (!P->device_ready) return fail(IFGF_EINVAL, "plan was built host-only");
  // The apply's workspace, carved from the static array in 256-byte aligned
  // regions: two cone-value buffers, the sorted densities, the sorted output.
  auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t need = 2 * up(P->ws_vbytes) + 2 * up(P->ws_pbytes);
  if (need > (int64_t)kStaticScratchBytes)
    return fail(IFGF_EINVAL, "ifgf_apply_noalloc: the plan's workspace (" +
                                 std::to_string(need) + " bytes) exceeds the static scratch of " +
                                 std::to_string((int64_t)kStaticScratchBytes) + " bytes");
  hipError_t e = hipSetDevice(P->device);
  void* base = nullptr;
  if (e == hipSuccess) e = static_scratch(&base);
  if (e == hipSuccess) {
    ApplyArgs A = P->A;
    char* p = (char*)base;
    A.vbuf[0] = p;
    A.vbuf[1] = p + up(P->ws_vbytes);
    A.dens_sorted = p + 2 * up(P->ws_vbytes);
    A.out_sorted = p + 2 * up(P->ws_vbytes) + up(P->ws_pbytes);
    e = launch_apply(A, P->p_s, P->p_ang, P->opts.precision, dens, out, P->stream, nullptr);
  }
  if (e != hipSuccess)
    return fail(IFGF_EHIP, std::string("apply_noalloc: ") + hipGetErrorString(e));
  return IFGF_OK;
}

ifgf_status ifgf_check(ifgf_plan_t P) {
  if (!P) return fail(IFGF_EINVAL, "null plan");
  if (!P->device_ready) return IFGF_OK;
  int flag = 0, zero = 0;
  hipError_t e = hipStreamSynchronize(P->stream);
  if (e == hipSuccess) e = hipMemcpy(&flag, P->A.err, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess && flag) e = hipMemcpy(P->A.err, &zero, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(IFGF_EHIP, std::string("check: ") + hipGetErrorString(e));
  if (flag) return fail(IFGF_ELOOKUP, "a cone look-up missed during apply");
  return IFGF_OK;
}

ifgf_status ifgf_profile(ifgf_plan_t P, int enable) {
  if (!P) return fail(IFGF_EINVAL, "null plan");
  P->profiling = enable != 0;
  return IFGF_OK;
}

ifgf_status ifgf_profile_read(ifgf_plan_t P, ifgf_stage_times* t, int reset) {
  if (!P || !t) return fail(IFGF_EINVAL, "null argument");
  hipError_t e = hipSuccess;
  if (P->prof_pending > 0) {
    e = hipStreamSynchronize(P->stream);
    for (int i = 0; e == hipSuccess && i < P->prof_pending; ++i) {
      float ms = 0;
      e = hipEventElapsedTime(&ms, P->prof_recs[i].a, P->prof_recs[i].b);
      if (e == hipSuccess) {
        P->prof_ms[P->prof_recs[i].stage] += ms;
        P->prof_launches[P->prof_recs[i].stage] += 1;
      }
    }
    P->prof_pending = 0;
  }
  if (e != hipSuccess) return fail(IFGF_EHIP, std::string("profile: ") + hipGetErrorString(e));
  for (int k = 0; k < IFGF_N_STAGES; ++k) {
    t->ms[k] = P->prof_ms[k];
    t->launches[k] = P->prof_launches[k];
    if (reset) {
      P->prof_ms[k] = 0;
      P->prof_launches[k] = 0;
    }
  }
  return IFGF_OK;
}

ifgf_status ifgf_set_stream(ifgf_plan_t P, void* s) {
  if (!P) return fail(IFGF_EINVAL, "null plan");
  P->stream = (hipStream_t)s;
  return IFGF_OK;
}

ifgf_status ifgf_plan_info(ifgf_plan_t P, ifgf_info* info) {
  if (!P || !info) return fail(IFGF_EINVAL, "null argument");
  *info = P->info;
  return IFGF_OK;
}

ifgf_status ifgf_cone_keys(ifgf_plan_t P, int step, uint64_t* keys, int64_t capacity) {
  if (!P || (!keys && capacity > 0)) return fail(IFGF_EINVAL, "null argument");
  if (!P->device_ready) return fail(IFGF_EINVAL, "plan was built host-only");
  if (step < 0 || step >= P->A.n_steps) return fail(IFGF_EINVAL, "step out of range");
  int64_t n = std::min<int64_t>(capacity, P->steps_h[step].ncones);
  if (n <= 0) return IFGF_OK;
  hipError_t e = hipSetDevice(P->device);
  if (e == hipSuccess)
    e = hipMemcpy(keys, P->steps_h[step].cone_key, sizeof(uint64_t) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(IFGF_EHIP, std::string("cone keys: ") + hipGetErrorString(e));
  return IFGF_OK;
}

ifgf_status ifgf_partition_counts(ifgf_plan_t P, int64_t* counts) {
  if (!P || !counts) return fail(IFGF_EINVAL, "null argument");
  partition_counts(P->m, counts);
  return IFGF_OK;
}

void ifgf_destroy(ifgf_plan_t P) { delete P; }

const char* ifgf_status_string(ifgf_status s) {
  static thread_local std::string buf;
  const char* base = "unknown status";
  switch (s) {
    case IFGF_OK: base = "ok"; break;
    case IFGF_EINVAL: base = "invalid argument"; break;
    case IFGF_ENOMEM: base = "out of memory"; break;
    case IFGF_EDUPLICATE: base = "duplicate points"; break;
    case IFGF_EHIP: base = "HIP error"; break;
    case IFGF_EUNSUPPORTED: base = "unsupported"; break;
    case IFGF_ELOOKUP: base = "cone look-up miss"; break;
  }
  buf = base;
  if (s != IFGF_OK && !g_err.empty()) buf += ": " + g_err;
  return buf.c_str();
}

}  // extern "C"
