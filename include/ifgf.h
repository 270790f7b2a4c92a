/*
 * ifgf.h -- C ABI of libifgf.so, the MI355X (gfx950) implementation of the
 * Interpolated Factored Green Function (IFGF) evaluation of the discrete
 * Helmholtz operator (Bauinger & Bruno, "Massively parallelized interpolated
 * factored Green function method", Section 2, eq. (field1)):
 *
 *     out_l = sum_{m != l} a_m exp(i kappa |x_l - x_m|) / (4 pi |x_l - x_m|),
 *     l = 1..N.
 *
 * Sign e^{+i kappa r}, the factor 1/(4 pi) included, the self term excluded.
 *
 * Conventions for every entry point:
 *   - Plain C types only; no C++ exception crosses the boundary.
 *   - Every function returns an ifgf_status; on error nothing is written to
 *     the caller's output and ifgf_status_string() describes the failure
 *     (for IFGF_EHIP it includes the HIP error of the failing call).
 *   - Points are FP64, N x 3 row-major, in host or device memory (device
 *     points are copied to the host, where the octree is built; a
 *     host_only plan needs host points).  Densities and outputs are DEVICE
 *     pointers on the plan's GPU.
 *   - Complex numbers are interleaved (re, im): complex128 (two doubles) in
 *     IFGF_FP64 mode, complex64 (two floats) in IFGF_FP32_MIXED and
 *     IFGF_FP32_BF16X3 modes.
 *   - Densities and outputs are laid out [n_rhs][N] in the caller's point
 *     order (RHS-major, point index fastest).
 */
#ifndef IFGF_H
#define IFGF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ifgf_plan_s* ifgf_plan_t; /* opaque, owned by the library */

typedef enum {
  IFGF_OK = 0,
  IFGF_EINVAL = 1,      /* n < 2, kappa < 0 or non-finite, kappa = 0
                           without a wavelength-free level rule (levels or
                           leaf_abs), p < 1, NaN/Inf coordinates, bad
                           options, null pointers */
  IFGF_ENOMEM = 2,      /* host or device allocation failed */
  IFGF_EDUPLICATE = 3,  /* two identical points: eq. (field1) is singular */
  IFGF_EHIP = 4,        /* a HIP runtime call failed */
  IFGF_EUNSUPPORTED = 5,/* (p_s, p_ang) without a compiled kernel, N >= 2^31,
                           too many levels */
  IFGF_ELOOKUP = 6      /* a cone look-up missed during apply (internal
                           consistency error; reported by ifgf_check) */
} ifgf_status;

typedef enum { IFGF_FP64 = 0, IFGF_FP32_MIXED = 1, IFGF_FP32_BF16X3 = 2 } ifgf_precision;

/* Options of a plan.  Obtain defaults with ifgf_default_opts(). */
typedef struct ifgf_opts {
  int precision;    /* ifgf_precision.  IFGF_FP32_MIXED: interpolation,
                       propagation and near field in FP32 complex; point and
                       box-centre geometry, cone selection, the phase
                       kappa*|x - x_c| (argument reduction) and the
                       centred-factor ratio in FP64.  IFGF_FP32_BF16X3: as
                       IFGF_FP32_MIXED, except that the wave-task
                       propagation kernels take the interpolation product
                       on BF16 matrix cores in three-term split form
                       (x = bf16(x) + bf16(x - bf16(x)) for both operands,
                       the low-by-low term dropped, FP32 accumulation;
                       about 2^-16 relative error per product; an addition
                       beyond the paper). */
  int n_rhs;        /* number of right-hand sides per apply, >= 1 */
  int leaf_grid[3]; /* cone-segment grid (n_s, n_theta, n_phi) at the leaf
                       level D; see grid_rule for the other levels.
                       {0,0,0} selects the default {2,4,8}. */
  int levels;       /* number of octree levels D of every instance; 0
                       selects D per instance by the level rule:
                       D = max(3, 1 + round(log2(H_1 / w))) with w = leaf_abs
                       if leaf_abs > 0, else w = leaf_size * lambda
                       (lambda = 2 pi / kappa); then, if leaf_max > 0, D
                       grows by one while H_1 / 2^(D-1) > leaf_max * lambda */
  int stages;       /* bit 0: near field (level-D neighbours, direct sum);
                       bit 1: far field (IFGF levels D..3).  0 means both. */
  int host_only;    /* 1: build the host octree only (no GPU used); only
                       ifgf_plan_info and ifgf_partition_counts may be
                       called on such a plan */
  int device;       /* HIP device ordinal; -1 uses the current device */
  void* stream;     /* hipStream_t used by ifgf_apply; NULL = null stream */
  int prop_kernel;  /* propagation kernel per level: 0 chooses by the mean
                       number of boxes sharing a parent cone index (>= 32:
                       four-wave matrix-core tasks; >= 4: one-wave
                       matrix-core tasks; else per-node), 1 forces the
                       per-node form, 2 the matrix-core block form, 3 the
                       one-wave task form, 4 the four-wave task form, 5 the
                       four-wave task form with smaller chunks (40 boxes;
                       four blocks per CU instead of three) */
  int lookup;       /* cone look-up: 0 dense tables where a level's table
                       (boxes x cone grid) has <= 2^28 entries, hash tables
                       elsewhere; 1 hash tables everywhere */
  int autotune;     /* 1: at plan time, time the five propagation kernels
                       on every level where the matrix-core forms apply and
                       keep the fastest (overrides prop_kernel there) */
  double cone_margin; /* a point within cone_margin cone widths of a cone
                       boundary also marks the adjacent cone relevant, so
                       that look-ups along other rounding paths never miss;
                       default 1e-9; 0 gives exactly the point-based
                       relevant cones of eq. (relevantconesegments) */
  double leaf_max;  /* per-instance accuracy control: cap on the leaf box
                       side in wavelengths (0: no cap).  The rounding of the
                       level rule puts leaves between 0.71 and 1.41 times
                       leaf_size; the method's error grows with the leaf
                       side (Section "Numerical error estimation"), and a
                       cap adds a level to an instance whose leaves would be
                       wider.  Ignored for kappa = 0. */
  double leaf_abs;  /* leaf box side in the points' length unit (0: use
                       leaf_size wavelengths).  The level rule for the
                       Laplace kernel (kappa = 0), which has no wavelength. */
  int grid_rule;    /* cone grid of the levels above the leaf: 0 doubles
                       every dimension per level up when kappa > 0 (the
                       phase varies over a box of side H_d at the scale
                       kappa H_d) and keeps the leaf grid at every level
                       when kappa = 0 (the analytic factor is then
                       scale-free in (s, theta, phi)); 1 always doubles;
                       2 always keeps the leaf grid.  One batched plan
                       cannot mix kappa = 0 and kappa > 0 under rule 0. */
  const char* tune_cache; /* path of the autotuner's cache file (NULL or
                       "": none).  With autotune = 1, a plan whose shape,
                       precision, RHS count and kernel build match a line
                       of the file takes the kernels recorded there instead
                       of timing them, and a plan that times them appends a
                       line. */
  int prop_tables;  /* plan-time tables of the matrix-core propagation (the
                       node geometry of every parent cone index and child
                       octant, which does not depend on the box): 0 builds
                       them for the steps nearest the leaves within four times
                       the bytes of one cone-value buffer (at least 1 GiB), 1 never,
                       2 for every step; 0 and 2 leave a tenth of the device
                       memory (at least 4 GiB) free.  Results are identical
                       either way. */
} ifgf_opts;

/* Size information about a plan (ifgf_plan_info). */
#define IFGF_MAX_LEVELS 24
typedef struct ifgf_info {
  int64_t n_points;       /* total points (all instances) */
  int n_instances;
  int max_levels;         /* max D over instances */
  int n_steps;            /* levels >= 3 handled on the GPU (= max D - 2) */
  int p_s, p_ang, n_rhs, precision;
  /* Per step l = D - d (l = 0 is the leaf level), summed over instances: */
  int64_t boxes[IFGF_MAX_LEVELS];      /* relevant boxes */
  int64_t cones[IFGF_MAX_LEVELS];      /* relevant cone segments */
  int64_t cousin_pairs[IFGF_MAX_LEVELS]; /* (target, cousin box) pairs */
  int64_t grid[IFGF_MAX_LEVELS];       /* cone grid size per box */
  int64_t prop_pairs[IFGF_MAX_LEVELS]; /* (parent-cone node, relevant child)
                                         evaluations of Propagation into
                                         step l (l >= 1) */
  int prop_mode[IFGF_MAX_LEVELS];      /* kernel of Propagation into step l:
                                         1 per-node, 2 matrix-core blocks,
                                         3 one-wave matrix-core tasks,
                                         4 four-wave matrix-core tasks,
                                         5 four-wave tasks, smaller chunks */
  float autotune_ms[IFGF_MAX_LEVELS][5]; /* autotuner timings of Propagation
                                         into step l, kernels 1..5 in order
                                         (0 when not tuned): the mean of two
                                         launches, or one launch for a form
                                         whose first launch took 1.5 times
                                         the best so far */
  int64_t leaf_pairs;     /* (leaf-cone node, source) evaluations of
                             LevelDEvaluations */
  int64_t near_pairs;     /* (target, source) near-field pairs, self included */
  int64_t device_bytes;   /* device memory held by the plan */
  double plan_seconds;    /* wall time of plan construction */
  int tune_cache_hit;     /* 1 when the kernels came from the tuning cache */
  int grid_doubling;      /* 1 when the cone grid doubles per level up */
  int64_t prop_table_bytes; /* device bytes of the propagation tables */
} ifgf_info;

/* Fill *opts with the defaults: FP64, 1 RHS, leaf grid {2,4,8}, automatic
 * D, both stages, device -1, null stream. */
ifgf_status ifgf_default_opts(ifgf_opts* opts);

/* Plan one instance (Section 2 of the paper: octree, relevant boxes,
 * neighbour and cousin lists, relevant cone segments; Morton ordering of
 * Section 3.2).  points: N x 3 FP64 array (host or device), copied.
 * kappa > 0 (kappa = 0, the Laplace kernel, needs opts.leaf_abs or
 * opts.levels through ifgf_plan_ex).
 * p_s, p_ang: Chebyshev points per cone in the radial and in each angular
 * variable (P = p_s * p_ang^2 interpolation points per cone); compiled
 * kernels exist for (3,5), (2,3) and (5,7).  leaf_size: leaf box side in
 * wavelengths (0.25 is typical).  Uses default options. */
ifgf_status ifgf_plan(ifgf_plan_t* plan, const double* points, int64_t n,
                      double kappa, int p_s, int p_ang, double leaf_size);

/* As ifgf_plan with explicit options (opts may be NULL for defaults). */
ifgf_status ifgf_plan_ex(ifgf_plan_t* plan, const double* points, int64_t n,
                         double kappa, int p_s, int p_ang, double leaf_size,
                         const ifgf_opts* opts);

/* Plan n_inst independent instances evaluated together by every apply
 * (each kernel launch processes all instances): the batched form of the
 * operator of eq. (field1), one independent sum per instance.  Instance i owns points
 * [offsets[i], offsets[i+1]) of `points` (host or device memory, as for
 * ifgf_plan; offsets, a host array, has n_inst+1
 * entries, offsets[0] = 0), wavenumber kappas[i].  Densities and outputs of
 * a batched apply are [n_rhs][N_total], N_total = offsets[n_inst], in that
 * concatenated order.  Interactions never cross instances. */
ifgf_status ifgf_plan_batched(ifgf_plan_t* plan, int n_inst,
                              const int64_t* offsets, const double* points,
                              const double* kappas, int p_s, int p_ang,
                              double leaf_size, const ifgf_opts* opts);

/* Evaluate out = A(densities) (eq. (field1)) on the plan's stream.
 * densities, out: device pointers, [n_rhs][N] interleaved complex of the
 * plan's precision (complex128 for IFGF_FP64, complex64 for
 * IFGF_FP32_MIXED and IFGF_FP32_BF16X3); out is overwritten.  Asynchronous with respect to the
 * host; one apply at a time per plan (not re-entrant).  A cone look-up that
 * misses (an internal consistency error) is skipped and only flagged: call
 * ifgf_check after the apply before trusting its result. */
ifgf_status ifgf_apply(ifgf_plan_t plan, const void* densities, void* out);

/* As ifgf_apply, through a HIP graph: the first call for a (densities,
 * out) pair captures the whole apply (every kernel launch of every level)
 * into a graph and instantiates it; later calls with the same pointers
 * replay it with one hipGraphLaunch on the plan's stream.  Other pointers
 * re-capture.  Profiling is not applied to graph launches. */
ifgf_status ifgf_apply_graph(ifgf_plan_t plan, const void* densities, void* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): as
 * ifgf_apply, but the apply's workspace (the two buffers of cone values of
 * consecutive levels, the densities and the output in sorted order) is a
 * static device array of the library, 256 MiB per GPU, held from the
 * library's first use on that GPU until the process ends, instead of the
 * plan's own buffers.  The call allocates nothing (no hipMalloc, no events)
 * and launches the same kernels as ifgf_apply on the plan's stream; every
 * workspace byte is written before it is read, so nothing is cleared
 * between calls.  A plan whose workspace exceeds 256 MiB is rejected with
 * IFGF_EINVAL.  All calls on one GPU share its array: calls that overlap in
 * time on the same GPU (other streams, other threads) race and must be
 * serialised by the caller.  Look-up misses are flagged as for ifgf_apply
 * (ifgf_check). */
ifgf_status ifgf_apply_noalloc(ifgf_plan_t plan, const void* densities, void* out);

/* Wait for the plan's stream and report whether any cone look-up of the
 * previous applies missed (IFGF_ELOOKUP); clears the flag. */
ifgf_status ifgf_check(ifgf_plan_t plan);

/* Change the stream used by later applies (hipStream_t; NULL = null stream). */
ifgf_status ifgf_set_stream(ifgf_plan_t plan, void* hip_stream);

/* Kernel stages timed by the profiler. */
typedef enum {
  IFGF_STAGE_PERMUTE_IN = 0,
  IFGF_STAGE_NEAR_FIELD = 1,
  IFGF_STAGE_LEAF = 2,          /* LevelDEvaluations */
  IFGF_STAGE_INTERPOLATION = 3, /* Interpolation(d), all levels */
  IFGF_STAGE_PROPAGATION = 4,   /* Propagation(d), per-node kernel levels */
  IFGF_STAGE_PERMUTE_OUT = 5,
  IFGF_STAGE_PROPAGATION_MFMA = 6, /* Propagation(d), matrix-core block levels */
  IFGF_STAGE_PROPAGATION_SMALL = 7, /* Propagation(d), wave-task matrix-core levels */
  IFGF_N_STAGES = 8
} ifgf_stage;

typedef struct ifgf_stage_times {
  double ms[IFGF_N_STAGES];        /* summed kernel durations (HIP events) */
  int64_t launches[IFGF_N_STAGES]; /* kernel launches timed */
} ifgf_stage_times;

/* Enable (1) or disable (0) timing of every kernel launch of later applies
 * with HIP events recorded on the plan's stream around each launch. */
ifgf_status ifgf_profile(ifgf_plan_t plan, int enable);

/* Wait for the plan's stream, add up the timed launches since the last
 * reset into *times, and reset the accumulators if reset != 0. */
ifgf_status ifgf_profile_read(ifgf_plan_t plan, ifgf_stage_times* times,
                              int reset);

/* Sizes and counts of the plan. */
ifgf_status ifgf_plan_info(ifgf_plan_t plan, ifgf_info* info);

/* Relevant cone segments of step l (level D - l): writes min(capacity,
 * info.cones[l]) keys box * grid[l] + gamma to the host array keys, in
 * ascending order (boxes in Morton order, the batched instances
 * concatenated; gamma = (i_s n_theta + i_theta) n_phi + i_phi). */
ifgf_status ifgf_cone_keys(ifgf_plan_t plan, int step, uint64_t* keys,
                           int64_t capacity);

/* Per point (caller order): the number of sources covered by the near-field
 * neighbour boxes (itself included) plus the points of every cousin box of
 * levels D..3.  Equals the instance's N for every point (the partition of
 * the sources of Section 2).  counts: host array of N_total int64. */
ifgf_status ifgf_partition_counts(ifgf_plan_t plan, int64_t* counts);

/* Release all memory of the plan (host and device).  NULL is ignored. */
void ifgf_destroy(ifgf_plan_t plan);

/* Human-readable text for a status, including the last HIP error text for
 * IFGF_EHIP.  Never NULL. */
const char* ifgf_status_string(ifgf_status status);

#ifdef __cplusplus
}
#endif

#endif /* IFGF_H */
