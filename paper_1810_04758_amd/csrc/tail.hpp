// tail.hpp -- brute-force tail of the level loop (few remaining queries
// against every point, with the whole GPU).
#pragma once

#include "kernels.hpp"

namespace knn {

struct TailState {
  unsigned __int128 A, B;  // inclusive (d2 bits, id) key interval while refining
  int32_t sh;              // the current round's sub-range width: 2^sh keys
  int32_t bsel, c_lo, c_hi, mode, fill;
};

struct TailArgs {
  const double* X;  // SoA coordinates in id order
  int64_t N;
  int32_t n;
  const int32_t* q_ids;  // the tail queries (point ids), A of them
  // external queries (a join of a query set with the indexed set): their
  // SoA coordinates QX[j*QN + id] by query id, and nothing excluded; NULL:
  // the queries are points of X and each excludes itself
  const double* QX;
  int64_t QN;
  int32_t A;
  int64_t top;  // bit pattern of the squared bounding-box diagonal >> 50
  int32_t K;
  int32_t cap;  // per-query survivor buffer entries (>= K)
  int32_t* out_ids;
  double* out_d;
  // carved from the scratch by tail_run
  TailState* state;
  uint32_t* hist;
  uint32_t* cnt;  // refinement: kTailSplit counts per query
  int32_t* flag;
  double* buf_d;
  int32_t* buf_i;
};

// Device scratch bytes tail_run needs for A queries.
size_t tail_state_bytes(int64_t A, int cap);
// Runs the whole tail on stream s; returns the number of refinement rounds.
// fixed_rounds >= 0: issue exactly that many refinement rounds with no host
// round trip (a replay of a recorded run; rounds beyond a query's need leave
// it unchanged); < 0: run until no query needs refinement.  Returns the rounds.
int tail_run(TailArgs a, char* scratch, hipStream_t s, int fixed_rounds = -1);

}  // namespace knn
