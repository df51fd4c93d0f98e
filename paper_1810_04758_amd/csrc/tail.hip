// tail.hip -- brute-force tail of the GPU-only join: the remedy the paper
// suggests for the GPU-Only long tail (Sec. 5.4, characterization of the
// search-distance expansion): once few queries remain, search them against
// every point instead of growing eps further.
//
// The few remaining queries are searched against all N points with the whole
// GPU: blocks cover (chunk of points) x (batch of QB queries); a thread keeps
// its points' coordinates in registers and loops over the batch, so every
// coordinate is read once per batch.  The selection is the grid kernel's, kept
// in global memory:
//   1. count pass: per-query histogram of log-spaced d^2 bins (16 octaves at 4
//      bins per octave, ending at the squared bounding-box diagonal; every
//      point is a candidate, so every query succeeds);
//   2. select: first bin whose cumulative count reaches K;
//   3. if it would overflow the per-query buffer, exact refinement of the key
//      (d^2, id) inside that bin: each round counts the keys of the interval
//      in 64 equal key sub-ranges (6 bits of the key per round) and keeps
//      the first where the count reaches K, one counting pass per round;
//   4. collect the survivors into the per-query buffer;
//   5. one wavefront per query ranks its survivors and writes the output row.
#pragma clang fp contract(off)

#include "tail.hpp"

namespace knn {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = kBlock * 8;      // points per block
constexpr int QB = 32;                   // queries per block
constexpr int TNB = 64;
constexpr int kTailShift = 50;
constexpr int kTailSplit = 64;     // key sub-ranges per refinement round
constexpr int kLog2TailSplit = 6;

__device__ __forceinline__ int tbitlen128(unsigned __int128 v) {
  const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
  return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}

enum Mode : int { kBin = 0, kRefine = 1, kKey = 2 };

__device__ __forceinline__ int tbin(double d2, int64_t top) {
  const int64_t k = (int64_t)((uint64_t)__double_as_longlong(d2) >> kTailShift) - top + (TNB - 1);
  return k < 0 ? 0 : (k > TNB - 1 ? TNB - 1 : (int)k);
}

template <int DIM>
__device__ __forceinline__ double tail_d2(const double* x, const double* qx) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double t = __dsub_rn(x[j], qx[j]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

// The batch's query coordinates and ids, staged in LDS.
struct QBatch {
  double x[QB][kMaxDims];
  int64_t id[QB];
  int nq;
};

__device__ __forceinline__ void load_batch(const TailArgs& a, QBatch& qb) {
  const int q0 = blockIdx.y * QB;
  const int nq = min(QB, a.A - q0);
  if (threadIdx.x == 0) qb.nq = nq;
  for (int i = threadIdx.x; i < nq; i += blockDim.x) {
    const int64_t id = a.q_ids[q0 + i];
    qb.id[i] = id;
    for (int j = 0; j < a.n; ++j)
      qb.x[i][j] = a.QX ? a.QX[(int64_t)j * a.QN + id] : a.X[(int64_t)j * a.N + id];
  }
}

// Coordinates of this thread's points (PPT of them, strided by the block,
// PPT * kBlock = kChunk), kept in registers.
template <int DIM, int PPT>
__device__ __forceinline__ void load_points(const TailArgs& a, int part, double (&px)[PPT][DIM],
                                            int64_t (&pid)[PPT]) {
  const int64_t p0 = (int64_t)blockIdx.x * kChunk + (int64_t)part * PPT * kBlock + threadIdx.x;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int64_t p = p0 + (int64_t)k * kBlock;
    pid[k] = p < a.N ? p : -1;
#pragma unroll
    for (int j = 0; j < DIM; ++j) px[k][j] = p < a.N ? a.X[(int64_t)j * a.N + p] : 0.0;
  }
}
template <int DIM>
constexpr int ppt() { return DIM <= 3 ? 8 : 4; }

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_tail_hist(const TailArgs a) {
  constexpr int PPT = ppt<DIM>();
  __shared__ QBatch qb;
  __shared__ uint32_t h[QB][TNB];
  for (int i = threadIdx.x; i < QB * TNB; i += blockDim.x) h[i / TNB][i % TNB] = 0;
  load_batch(a, qb);
  __syncthreads();
  for (int part = 0; part < 8 / PPT; ++part) {
    double px[PPT][DIM];
    int64_t pid[PPT];
    load_points<DIM, PPT>(a, part, px, pid);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (pid[k] < 0) continue;
      for (int i = 0; i < qb.nq; ++i) {
        if (!a.QX && pid[k] == qb.id[i]) continue;
        atomicAdd(&h[i][tbin(tail_d2<DIM>(px[k], qb.x[i]), a.top)], 1u);
      }
    }
  }
  __syncthreads();
  const int q0 = blockIdx.y * QB;
  for (int e = threadIdx.x; e < qb.nq * TNB; e += blockDim.x) {
    const uint32_t v = h[e / TNB][e % TNB];
    if (v) atomicAdd(&a.hist[(int64_t)(q0 + e / TNB) * TNB + e % TNB], v);
  }
}

// One thread per query: selected bin, counts, mode and (for refinement) the
// exact key interval of the selected bin.
__global__ void k_tail_select(const TailArgs a) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.A) return;
  TailState& st = a.state[qi];
  int cum = 0, bsel = TNB - 1, c_lo = 0, c_hi = 0;
  for (int b = 0; b < TNB; ++b) {
    const int h = (int)a.hist[qi * TNB + b];
    if (cum + h >= a.K) {
      bsel = b;
      c_lo = cum;
      c_hi = cum + h;
      break;
    }
    cum += h;
  }
  st.bsel = bsel;
  st.c_lo = c_lo;
  st.c_hi = c_hi;
  st.fill = 0;
  if (c_hi <= a.cap) {
    st.mode = kBin;
  } else {
    st.mode = kRefine;
    atomicAdd(&a.flag[0], 1);
    // d2 bit patterns of bin b (unclamped) are [v << shift, ((v+1) << shift) - 1],
    // v = top - (TNB-1) + b; bin 0 also holds everything below, the last bin
    // everything above
    const int64_t v = a.top - (TNB - 1) + bsel;
    const uint64_t lo_bits = bsel == 0 ? 0ull : ((uint64_t)v << kTailShift);
    const uint64_t hi_bits =
        bsel == TNB - 1 ? ~0ull : ((((uint64_t)(v + 1)) << kTailShift) - 1ull);
    st.A = (unsigned __int128)lo_bits << 32;
    st.B = ((unsigned __int128)hi_bits << 32) | 0xFFFFFFFFu;
  }
}

// Per query in refinement: the width 2^sh of the round's kTailSplit equal key
// sub-ranges of [A, B] (the last one may be partial), and cleared counts.
__global__ void k_tail_split(const TailArgs a) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.A) return;
  TailState& st = a.state[qi];
  if (st.mode != kRefine) return;
  const int sh = tbitlen128(st.B - st.A) - kLog2TailSplit;
  st.sh = sh < 0 ? 0 : sh;
  for (int i = 0; i < kTailSplit; ++i) a.cnt[(int64_t)qi * kTailSplit + i] = 0;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_tail_refine_count(const TailArgs a) {
  constexpr int PPT = ppt<DIM>();
  __shared__ QBatch qb;
  __shared__ uint32_t cs[QB][kTailSplit];
  __shared__ int refining[QB], ssh[QB];
  __shared__ unsigned __int128 sA[QB], sB[QB];
  __shared__ int any;
  const int q0 = blockIdx.y * QB;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < QB; i += blockDim.x) {
    const bool r = q0 + i < a.A && a.state[q0 + i].mode == kRefine;
    refining[i] = r;
    if (r) {
      any = 1;
      sA[i] = a.state[q0 + i].A;
      sB[i] = a.state[q0 + i].B;
      ssh[i] = a.state[q0 + i].sh;
    }
  }
  for (int e = threadIdx.x; e < QB * kTailSplit; e += blockDim.x) cs[e / kTailSplit][e % kTailSplit] = 0;
  load_batch(a, qb);
  __syncthreads();
  if (!any) return;
  for (int part = 0; part < 8 / PPT; ++part) {
    double px[PPT][DIM];
    int64_t pid[PPT];
    load_points<DIM, PPT>(a, part, px, pid);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (pid[k] < 0) continue;
      for (int i = 0; i < qb.nq; ++i) {
        if (!refining[i] || (!a.QX && pid[k] == qb.id[i])) continue;
        const double d2 = tail_d2<DIM>(px[k], qb.x[i]);
        const unsigned __int128 key =
            ((unsigned __int128)(uint64_t)__double_as_longlong(d2) << 32) | (uint32_t)pid[k];
        if (key >= sA[i] && key <= sB[i])  // (B - A) >> sh < kTailSplit
          atomicAdd(&cs[i][(int)((key - sA[i]) >> ssh[i])], 1u);
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < qb.nq * kTailSplit; e += blockDim.x) {
    const uint32_t v = cs[e / kTailSplit][e % kTailSplit];
    if (v) atomicAdd(&a.cnt[(int64_t)(q0 + e / kTailSplit) * kTailSplit + e % kTailSplit], v);
  }
}

__global__ void k_tail_refine_update(const TailArgs a) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.A) return;
  TailState& st = a.state[qi];
  if (st.mode != kRefine) return;
  // the first sub-range where the count (c_lo below A) reaches K
  const uint32_t* c = a.cnt + (int64_t)qi * kTailSplit;
  int cum = st.c_lo;
  int b = 0;
  for (; b < kTailSplit; ++b) {
    if (cum + (int)c[b] >= a.K) break;
    cum += (int)c[b];
  }
  if (b == kTailSplit) {
    // the counts of [A, B] always reach K; the passes disagreed: stop here
    // and report (the query keeps its interval)
    st.mode = kKey;
    atomicAdd(&a.flag[1], 1);
    return;
  }
  const unsigned __int128 nA = st.A + ((unsigned __int128)b << st.sh);
  const unsigned __int128 nB = nA + (((unsigned __int128)1 << st.sh) - 1);
  st.A = nA;
  if (nB < st.B) st.B = nB;
  st.c_hi = cum + (int)c[b];
  st.c_lo = cum;
  // a single-key interval holds at most one candidate, so this ends
  if (st.c_hi <= a.cap || st.A == st.B)
    st.mode = kKey;
  else
    atomicAdd(&a.flag[0], 1);
}

template <int DIM>
__global__ void __launch_bounds__(kBlock) k_tail_collect(const TailArgs a) {
  constexpr int PPT = ppt<DIM>();
  __shared__ QBatch qb;
  __shared__ int smode[QB], sbsel[QB];
  __shared__ unsigned __int128 sB[QB];
  const int q0 = blockIdx.y * QB;
  for (int i = threadIdx.x; i < QB; i += blockDim.x) {
    if (q0 + i < a.A) {
      smode[i] = a.state[q0 + i].mode;
      sbsel[i] = a.state[q0 + i].bsel;
      sB[i] = a.state[q0 + i].B;
    }
  }
  load_batch(a, qb);
  __syncthreads();
  for (int part = 0; part < 8 / PPT; ++part) {
    double px[PPT][DIM];
    int64_t pid[PPT];
    load_points<DIM, PPT>(a, part, px, pid);
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (pid[k] < 0) continue;
      for (int i = 0; i < qb.nq; ++i) {
        if (!a.QX && pid[k] == qb.id[i]) continue;
        const double d2 = tail_d2<DIM>(px[k], qb.x[i]);
        bool acc;
        if (smode[i] == kBin)
          acc = tbin(d2, a.top) <= sbsel[i];
        else
          acc = (((unsigned __int128)(uint64_t)__double_as_longlong(d2) << 32) |
                 (uint32_t)pid[k]) <= sB[i];
        if (acc) {
          TailState& st = a.state[q0 + i];
          const int slot = atomicAdd(&st.fill, 1);
          if (slot < a.cap) {
            a.buf_d[(int64_t)(q0 + i) * a.cap + slot] = d2;
            a.buf_i[(int64_t)(q0 + i) * a.cap + slot] = (int32_t)pid[k];
          }
        }
      }
    }
  }
}

// One wavefront per query: rank every survivor among the survivors in
// (d2, id) order; ranks below K go to the output row of the query.
__global__ void k_tail_finish(const TailArgs a) {
  const int qi = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (qi >= a.A) return;
  const int c = min(a.state[qi].fill, a.cap);
  const int64_t row = a.q_ids[qi];
  const double* bd = a.buf_d + (int64_t)qi * a.cap;
  const int32_t* bi = a.buf_i + (int64_t)qi * a.cap;
  for (int s = lane; s < c; s += 64) {
    const double da = bd[s];
    const int32_t ia = bi[s];
    int rank = 0;
    for (int s2 = 0; s2 < c; ++s2) {
      const double db = bd[s2];
      const int32_t ib = bi[s2];
      rank += (db < da || (db == da && ib < ia)) ? 1 : 0;
    }
    if (rank < a.K) {
      a.out_ids[row * a.K + rank] = ia;
      a.out_d[row * a.K + rank] = sqrt(da);
    }
  }
}

}  // namespace

size_t tail_state_bytes(int64_t A, int cap) {
  return (size_t)A * (sizeof(TailState) + TNB * 4 + kTailSplit * 4 + (size_t)cap * 12) + 6 * 256;
}

#define LAUNCH_DIM(kern, grid, args)                                           \
  do {                                                                         \
    switch ((args).n) {                                                        \
      case 2: kern<2><<<grid, kBlock, 0, s>>>(args); break;                    \
      case 3: kern<3><<<grid, kBlock, 0, s>>>(args); break;                    \
      case 4: kern<4><<<grid, kBlock, 0, s>>>(args); break;                    \
      case 5: kern<5><<<grid, kBlock, 0, s>>>(args); break;                    \
      case 6: kern<6><<<grid, kBlock, 0, s>>>(args); break;                    \
      default: throw Error(KNN_EINVAL, "dims out of range");                   \
    }                                                                          \
  } while (0)

int tail_run(TailArgs a, char* scratch, hipStream_t s, int fixed_rounds) {
  // carve the scratch: state, hist, cnt, flag, buffers
  char* p = scratch;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return r;
  };
  a.state = reinterpret_cast<TailState*>(take((size_t)a.A * sizeof(TailState)));
  a.hist = reinterpret_cast<uint32_t*>(take((size_t)a.A * TNB * 4));
  a.cnt = reinterpret_cast<uint32_t*>(take((size_t)a.A * kTailSplit * 4));
  a.flag = reinterpret_cast<int32_t*>(take(16));
  a.buf_d = reinterpret_cast<double*>(take((size_t)a.A * a.cap * 8));
  a.buf_i = reinterpret_cast<int32_t*>(take((size_t)a.A * a.cap * 4));
  launch_zero(a.hist, (size_t)a.A * TNB * 4, s);
  const dim3 grid((unsigned)ceil_div(a.N, kChunk), (unsigned)ceil_div(a.A, QB));
  LAUNCH_DIM(k_tail_hist, grid, a);
  KNN_LAUNCHED();
  const int sb = (int)ceil_div(a.A, kBlock);
  launch_zero(a.flag, 16, s);
  k_tail_select<<<sb, kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  int32_t nref = 0;
  const bool fixed = fixed_rounds >= 0;
  if (fixed) {
    nref = fixed_rounds;
  } else {
    KNN_HIP(hipMemcpyAsync(&nref, a.flag, 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
  }
  int rounds = 0;
  while (fixed ? rounds < fixed_rounds : nref > 0) {
    k_tail_split<<<sb, kBlock, 0, s>>>(a);
    KNN_LAUNCHED();
    LAUNCH_DIM(k_tail_refine_count, grid, a);
    KNN_LAUNCHED();
    launch_zero(a.flag, 4, s);
    k_tail_refine_update<<<sb, kBlock, 0, s>>>(a);
    KNN_LAUNCHED();
    if (!fixed) {
      int32_t fl[2] = {0, 0};
      KNN_HIP(hipMemcpyAsync(fl, a.flag, 8, hipMemcpyDeviceToHost, s));
      KNN_HIP(hipStreamSynchronize(s));
      nref = fl[0];
      KNN_CHECK(fl[1] == 0, KNN_EINTERNAL, "tail refinement: the counting passes disagreed");
    }
    ++rounds;
    KNN_CHECK(rounds < 200, KNN_EINTERNAL, "tail refinement did not converge");
  }
  LAUNCH_DIM(k_tail_collect, grid, a);
  KNN_LAUNCHED();
  k_tail_finish<<<(unsigned)ceil_div(a.A, 4), kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  return rounds;
}

}  // namespace knn
