// Host-side state of a batched solver (shared by the solve loop and the
// subspace-recycling entry point).
#pragma once

#include <vector>

#include "common.h"
#include "solver.h"

struct dd_solver {
  int nb = 0;
  dd_solver_opts o{};
  int R = 1;          // field elements per thread
  int nchunks = 0;
  int ncu = 1;        // compute units of the device
  std::vector<const fdfd_op*> ops;
  std::vector<ProbDesc> hdesc;
  std::vector<int> ksetup;  // augmenting columns given per problem
  ProbDesc* ddesc = nullptr;
  int* blk2prob = nullptr;
  const void** dU = nullptr;  // device array of nb pointers for set_subspace
  PlanDev P{};
  std::vector<void*> allocs;
  size_t bytes = 0;       // device workspace of the solver (owned or the caller's)
  bool owns_workspace = true;
  // fused Arnoldi sweep: on when cgs_passes = 1 and kmax + m + 1 <= 128
  bool fused = false;
  std::vector<FusedTile> htiles;
  FusedTile* dtiles = nullptr;
  int* pinned = nullptr;     // 2 status snapshots + 1 final
  double* pinnedD = nullptr;
  unsigned long long* pinnedK = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool has_subspace = false;
  // the basis slots and small matrices hold the last cycle of a solve (for
  // dd_solver_recycle) until set_subspace or the autotuner overwrites them
  bool cycle_valid = false;
  // live kernel timing (dd_solver_profile): event pairs around the three
  // streaming sweeps of every Arnoldi step, read back at each host sync
  bool prof = false;
  std::vector<hipEvent_t> pev;
  std::vector<int> pkind;
  int pused = 0;
  dd_kernel_stats ks{};
  // solve controls (pinned host staging, device copy)
  double* hctl = nullptr;
  double* dctl = nullptr;
  // HIP graphs of groups of check_every Arnoldi steps, captured on a private
  // stream on first use and replayed on the caller's stream
  hipStream_t cap = nullptr;
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs;
  // diagonal preconditioner buffers per problem (FP64 and FP32 copies)
  struct PcBuf { double2 *pl64, *pr64; float2 *pl32, *pr32; };
  std::vector<PcBuf> pcbuf;
};
