// Batched complex LU (row-major, pivoting through a row map) -- host API.
#pragma once

#include <vector>

#include "common.hpp"

namespace nep {

constexpr int kLuMaxJB = 128;
constexpr int kSolveBlkLu = 64;  // diagonal-block size of the stored inverses (the solve's block)
constexpr int kPart0Cols = 64;   // trailing columns updated first in each step (the next panel)
// small panels (at most 256 rows left) in a step before they take the
// 256-thread groups, by default
constexpr int kSmallPanelsMin = 512;
// plans whose matrices all have at least this many rows take 128-wide panels
constexpr int kLuWideMinN = 2048;

// Launch plan of a (possibly ragged) batch: matrices sorted by n, descending.
struct LuPlan {
  struct Step {
    int k0, nact;
    // matrices [0, nwide) have more than one panel row per thread; the rest
    // take the single-row panel.  Within [0, nwide) the matrices of more
    // than 2048 and 1024 rows left end at n8 and n4: each range takes the
    // rows per thread (and with it the leaf width and the rounding) the
    // matrix would get alone, so a matrix's panel depends on that matrix
    // only, not on its batch
    int nwide, n8, n4;
    // matrices [nsmall, nact) have at most 256 rows left: with enough of them
    // (complex FP32), a 256-thread panel group each, two per CU
    int nsmall;
    // tiles of the U12 product and of the trailing update; part 0 is the
    // first tile column (it holds the next panel), part 1 the rest
    int off_trsm[2], tot_trsm[2];
    int off_gemm[2], tot_gemm[2];
  };
  int jb = 128, prec = NEP_PREC_C32_IR64, nmat = 0, nmax = 0;
  // complex FP32: a step's small panels take the 256-thread groups when at
  // least small_min of them share the step (0: always; INT_MAX: never);
  // either group size gives the same bits, so this is a pure launch-shape knob
  int small_min = kSmallPanelsMin;
  // look-ahead fork point of the rest of a step's update: 1 as soon as the
  // panel is done, 0 after the first columns' update, -1 built in (1 for
  // 64-wide complex FP32 panels, else 0); a pure scheduling knob
  int early_fork = -1;
  std::vector<Step> steps;
  std::vector<int> prefix;  // uploaded once; offsets above index into it
  std::vector<int> nvec;    // sizes of the sorted matrices
  // jb_force: the panel width (64 or 128), 0 for the built-in choice
  void build(const std::vector<MatDesc>& sorted, int prec, int jb_force = 0);
};

// Event timing of the trailing-update GEMM launches (kind 0: c64, 1: c128).
struct KernelProf {
  bool on = false;
  struct Rec {
    int kind;
    hipEvent_t e0, e1;
    double flops;
  };
  std::vector<Rec> recs;
  void add(int kind, hipEvent_t a, hipEvent_t b, double f) { recs.push_back(Rec{kind, a, b, f}); }
};
KernelProf& kernel_prof();

int lu_jb(int prec, int nmin);
hipError_t lu_configure();

// Linv: workspace of 2 * nmat * kLuMaxJB^2 elements (inverses of the L11 blocks,
// one half per step parity).
// Dinv/dinv_off: per matrix, the inverses of the 64 x 64 diagonal blocks of L
// and U ([blk][0: L, 1: U][64][64]), written as the panels complete.
// Streams and events of the look-ahead schedule: the next panel runs on aux
// while the rest of the trailing update runs on the caller's stream, and the
// inverses of the U blocks run on side.  nullptr streams: no overlap.  All
// streams keep the default priority.
struct LuStreams {
  hipStream_t aux = nullptr, side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_side[2] = {nullptr, nullptr}, ev_side_done = nullptr;
};

// arrivals: nmat ints, zero before the first call (left zero by every call):
// per-matrix arrival counts of the fused first-columns update.
// rows_alt: rows_total ints, the second row-map buffer of the look-ahead
// schedule (the final map is always left in rows).
template <typename P>
hipError_t lu_run(const LuPlan& plan, const MatDesc* d_md, const int* d_prefix, cx<P>* T, int* rows, int* rows_alt,
                  int rows_total, int* info, const int* skip, cx<P>* Linv, cx<P>* Dinv, const long long* dinv_off,
                  int* arrivals, hipStream_t st, const LuStreams& ls);

}  // namespace nep
