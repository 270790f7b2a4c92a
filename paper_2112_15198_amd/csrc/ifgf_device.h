// ifgf_device.h -- device-side views of a plan, shared by the kernels and
// the host code that launches them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifgf {

static constexpr unsigned long long kEmptyKey = ~0ull;
static constexpr int kMaxRhs = 4;  // right-hand sides handled per apply

// First-kind Chebyshev nodes t_j = cos((2j+1) pi / (2n)) on [-1, 1] and the
// Lagrange product weights w_j = 1 / prod_{m != j} (t_j - t_m), radial (s)
// and angular (a).
struct ChebConst {
  double ts[8], ws[8], ta[8], wa[8];
};

// One tree level, counted from the leaf (step l = D - d), all instances.
struct StepDev {
  int64_t nb;                 // relevant boxes
  const double* center;       // 3 per box
  const int* inst;            // instance of each box
  const int* first;           // first point (sorted order)
  const int* count;           // points per box
  const int* child;           // 8 per box: children at step l-1, or -1
  const int64_t* cous_begin;  // cousin CSR
  const int* cous;
  const int* pt_box;          // per point: its box at this step, or -1
  const double* inst_h;       // per instance: h = (sqrt 3 / 2) H_d
  const double* inst_H;       // per instance: box side H_d
  // Cone grid (identical for every instance at a given step).
  int ns, nt, np;
  int64_t ngrid;              // ns * nt * np
  double ds, dt, dp;          // cone widths in s, theta, phi
  const double* s_node;       // ns * P_s node values of s
  const double* t_node;       // nt * P_ang (sin, cos) of theta at the nodes
  const double* p_node;       // np * P_ang (sin, cos) of phi at the nodes
  double rds, rdt, rdp;       // 1/ds, 1/dt, 1/dp
  const double* t_bnd;        // (cos, sin) of the theta boundaries i dt, i = 0..nt
  const double* p_bnd;        // (cos, sin) of the phi boundaries i dp, i = 0..np
  // Relevant cone segments, sorted by key = box * ngrid + gamma (the order
  // "box Morton order, then radial, elevation, azimuth").
  int64_t ncones;
  const unsigned long long* cone_key;
  const unsigned long long* hkey;  // open-addressing table key -> slot
  const int* hval;
  unsigned long long hmask;
  const int* table;           // dense key -> slot table (nb * ngrid), or null
  // Propagation into this step, grouped: the relevant cones sorted by
  // (instance, gamma, box) and cut into chunks of boxes sharing one gamma,
  // whose node geometry is computed once per chunk.
  int prop_grouped;           // kernel: kPropNode .. kPropLean
  int64_t nchunks;
  const int* gslot;           // slots in (instance, gamma, box) order
  const int64_t* chunk_start; // first index into gslot of each chunk
  const int* chunk_len;       // boxes in each chunk (<= chunk_boxes())
  int64_t nschunks;           // the same order cut into chunks of at most
  const int64_t* schunk_start; // small_chunk_boxes(nrhs, 1) boxes (one wave)
  const int* schunk_len;
  int64_t nmchunks;           // ... and of small_chunk_boxes(nrhs, kMediumWaves)
  const int64_t* mchunk_start;
  const int* mchunk_len;
  int64_t nlchunks;           // ... and of small_chunk_boxes(nrhs, kMediumWaves, kLeanBoxes)
  const int64_t* lchunk_start;
  const int* lchunk_len;
  // Groups: the runs of gslot sharing (instance, gamma).  The plan-time
  // table holds the box-independent record of every (group, octant)
  // (prop_table_record_bytes each, group-major), or is null.
  int64_t ngroups;
  const int64_t* group_first; // first index into gslot of each group
  const int* schunk_group;    // group of each one-wave chunk
  const int* mchunk_group;    // group of each kMediumWaves-wave chunk
  const int* lchunk_group;    // group of each lean kMediumWaves-wave chunk
  unsigned char* prop_table;
};

// Propagation kernels of a level: per node, matrix-core blocks, one-wave
// matrix-core tasks, kMediumWaves-wave matrix-core tasks, and the same with
// chunks of kLeanBoxes boxes per wave (smaller blocks, four per CU).
enum { kPropNode = 0, kPropGrouped = 1, kPropSmall = 2, kPropMedium = 3, kPropLean = 4,
       kPropKinds = 5 };
static constexpr int kMediumWaves = 4;
static constexpr int kTaskBoxes = 16;  // boxes per wave of a task chunk (one RHS)
static constexpr int kLeanBoxes = 10;  // ... of a lean task chunk

// Largest P = P_s P_ang^2 with a matrix-core propagation kernel.
static constexpr int kMfmaMaxP = 125;

// Boxes per chunk of the grouped (matrix-core) propagation: kSubChunks
// sub-chunks of 32 (FP32) or 16 (FP64) GEMM columns.
static constexpr int kSubChunks = 8;
int chunk_boxes(int precision, int nrhs);
// Boxes per chunk of the wave-task matrix-core propagation: per_wave boxes
// per wave with one RHS (kTaskBoxes: 16 GEMM columns), divided by kMaxRhs
// with several.
int small_chunk_boxes(int nrhs, int waves, int per_wave = kTaskBoxes);

// Everything a kernel needs; passed by value (small), the per-step views
// live in device memory.
struct ApplyArgs {
  int64_t n;                  // points, all instances
  int nrhs;
  int n_steps;
  int stages;                 // bit 0 near field, bit 1 far field
  const double* x;            // sorted coordinates
  const double* y;
  const double* z;
  const float4* q_leaf;       // FP32 modes: per sorted point (x - c, |x - c|^2),
                              // c the centre of its leaf box; null in FP64 mode
  const int* perm;            // sorted index -> caller index
  const double* inst_kappa;
  const int64_t* nbr_begin;   // level-D neighbour CSR
  const int* nbr;
  const StepDev* step;        // device array of n_steps views
  const StepDev* step_host;   // the same views in host memory (launch sizes)
  ChebConst cheb;
  int* err;                   // set when a cone look-up misses
  void* dens_sorted;          // [N][nrhs] complex, sorted order
  void* out_sorted;           // [N][nrhs] complex, sorted order
  void* vbuf[2];              // cone values of two consecutive levels
};

struct MarkArgs {
  unsigned long long* tab;
  unsigned long long mask;
  unsigned int* count;
  int* overflow;
  double margin;              // in cone widths
};

// Records a HIP event pair around each kernel launch of an apply.
struct Profiler {
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  Rec* recs = nullptr;  // pool
  int n = 0, cap = 0;
  hipError_t begin(int stage, hipStream_t st) {
    if (n >= cap) return hipErrorOutOfMemory;
    recs[n].stage = stage;
    return hipEventRecord(recs[n].a, st);
  }
  hipError_t end(hipStream_t st) { return hipEventRecord(recs[n++].b, st); }
};

hipError_t launch_fill_u64(unsigned long long* p, int64_t n,
                           unsigned long long v, hipStream_t st);
hipError_t launch_mark(const ApplyArgs& A, int l, int ps, int pa,
                       const MarkArgs& M, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
hipError_t launch_scatter_table(const unsigned long long* keys, int64_t n,
                                int* table, hipStream_t st);
hipError_t launch_compact(const unsigned long long* tab, int64_t cap,
                          unsigned long long* out, unsigned int* counter,
                          hipStream_t st);
hipError_t launch_build_lookup(const unsigned long long* keys, int64_t n,
                               unsigned long long* tab, int* val,
                               unsigned long long mask, int* overflow,
                               hipStream_t st);
hipError_t launch_group_keys(const unsigned long long* keys, int64_t n, unsigned long long ng,
                             const int* inst, unsigned long long* gk, int* idx,
                             hipStream_t st);
hipError_t sort_pairs(const unsigned long long* keys_in, unsigned long long* keys_out,
                      const int* vals_in, int* vals_out, int64_t n, int end_bit, void* scratch,
                      size_t* scratch_bytes, hipStream_t st);
hipError_t sort_keys(unsigned long long* keys, unsigned long long* tmp,
                     int64_t n, int end_bit, void* scratch,
                     size_t* scratch_bytes, hipStream_t st);
// Bytes of one (group, octant) record of a propagation table.
int prop_table_record_bytes(int ps, int pa, int precision);
// Fill the propagation table of step l + 1 (every group, every octant).
hipError_t launch_prop_table(const ApplyArgs& A, int l, int ps, int pa, int precision,
                             int64_t ngroups, hipStream_t st);
// One Propagation launch (step l -> l + 1) with kernel `kind` (kPropNode ..
// kPropLean), for timing at plan time;
// precision 0 FP64, 1 FP32-mixed, 2 FP32 with the three-term BF16 product.
hipError_t launch_prop_level(const ApplyArgs& A, int l, int ps, int pa,
                             int precision, int kind, hipStream_t st);
// The allocation-free apply's workspace: a static device array of
// kStaticScratchBytes per GPU.  *ptr receives its device address on the
// current device (looked up on the first call per device).
static constexpr size_t kStaticScratchBytes = size_t(256) << 20;
static constexpr int kMaxDevices = 64;
hipError_t static_scratch(void** ptr);
hipError_t launch_apply(const ApplyArgs& A, int ps, int pa, int precision,
                        const void* dens_user, void* out_user, hipStream_t st,
                        Profiler* prof);

}  // namespace ifgf
