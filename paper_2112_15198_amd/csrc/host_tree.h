// host_tree.h -- host-side octree of one or several IFGF instances.
//
// Builds, per instance, the box octree of Section 2 (half-open cubes, levels
// 1..D), the Morton order of points and boxes (Section 3.2), the level-D
// neighbour lists and the cousin lists of levels 3..D
// (eq. defneighboursandcousins), and merges the instances into one global
// index space per level counted from the leaf (step l = D_i - d), which is the
// layout the device kernels work on.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ifgf {

// One octree level of one instance (local indices).
struct TreeLevel {
  std::vector<uint64_t> key;    // Morton key of each relevant box, ascending
  std::vector<int64_t> first;   // first point (local sorted index)
  std::vector<int32_t> count;   // number of points
  std::vector<int32_t> k;       // multi-index, 3 per box
  std::vector<int32_t> parent;  // index in level d-1 (-1 at d = 1)
  std::vector<int32_t> child;   // 8 per box: index in level d+1 or -1
  std::vector<int64_t> cous_begin;  // cousin CSR (levels >= 3 only)
  std::vector<int32_t> cous;
};

struct InstanceTree {
  int64_t n = 0;          // points of this instance
  int64_t offset = 0;     // global offset of its points
  double kappa = 0;
  int D = 0;
  double H1 = 0;
  double corner[3] = {0, 0, 0};
  std::vector<int64_t> order;          // local sorted index -> local user index
  std::vector<double> xs[3];           // sorted coordinates
  std::vector<TreeLevel> lev;          // lev[d], d = 1..D (lev[0] unused)
  std::vector<int64_t> nbr_begin;      // level-D neighbour CSR (self included)
  std::vector<int32_t> nbr;
};

// Global, instance-merged arrays for the device (one entry per step).
struct MergedStep {
  int64_t nb = 0;
  std::vector<double> center;        // 3 per box
  std::vector<int32_t> inst;         // instance id per box
  std::vector<int32_t> first;        // first point (global sorted index)
  std::vector<int32_t> count;
  std::vector<int32_t> child;        // 8 per box, index at step l-1 (l >= 1)
  std::vector<int64_t> cous_begin;   // nb + 1
  std::vector<int32_t> cous;         // global box indices at this step
  std::vector<int32_t> pt_box;       // per global sorted point: box or -1
  std::vector<double> inst_h;        // per instance: h = (sqrt 3 / 2) H_d at this step
  std::vector<double> inst_H;        // per instance: H_d
};

struct Merged {
  int64_t n = 0;
  int n_inst = 0;
  int n_steps = 0;                    // max D - 2
  int max_D = 0;
  std::vector<int64_t> inst_offset;   // n_inst + 1
  std::vector<double> inst_kappa;
  std::vector<int32_t> inst_D;
  std::vector<double> xs[3];          // sorted coordinates
  std::vector<int32_t> perm;          // global sorted -> global user index
  std::vector<MergedStep> step;       // step[l], l = 0..n_steps-1
  std::vector<int64_t> nbr_begin;     // leaf-level neighbour CSR (global)
  std::vector<int32_t> nbr;
  int64_t near_pairs = 0;
};

// How the number of levels D of an instance is chosen: `levels` if > 0,
// else D = max(3, 1 + round(log2(H_1 / w))) with w = leaf_abs if > 0, else
// w = leaf_size wavelengths; then, when leaf_max > 0 and kappa > 0, D grows
// while the leaf side H_1 / 2^(D-1) exceeds leaf_max wavelengths.
struct LevelRule {
  int levels = 0;
  double leaf_size = 0.25;
  double leaf_max = 0;
  double leaf_abs = 0;
};

// Returns 0 on success, else an ifgf_status code; msg receives details.
int build_instance(const double* pts, int64_t n, double kappa,
                   const LevelRule& rule, InstanceTree& t, std::string& msg);

void build_lists(InstanceTree& t, int threads);

int merge_instances(std::vector<InstanceTree>& trees, Merged& m,
                    std::string& msg);

// Per point (global user order) near-field + cousin source counts.
void partition_counts(const Merged& m, int64_t* counts);

int default_threads();

}  // namespace ifgf
