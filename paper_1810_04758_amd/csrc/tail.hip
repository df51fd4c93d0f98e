// tail.hip -- brute-force tail of the GPU-only join (the remedy the paper
// suggests for the GPU-Only long tail, Sec. 5.3.8: once few queries remain,
// search them against every point instead of growing eps further).
//
// The few remaining queries are searched against all N points with the whole
// GPU: blocks cover (chunk of points) x (query).  The selection is the same as
// in the grid kernel, but kept in global memory:
//   1. count pass: per-query histogram of log-spaced d^2 bins (16 octaves at 4
//      bins per octave, ending at the squared bounding-box diagonal; every
//      point is a candidate, so every query succeeds);
//   2. select: first bin whose cumulative count reaches K;
//   3. if it would overflow the per-query buffer, exact bisection of the key
//      (d^2, id) inside that bin, one counting pass per round;
//   4. collect the survivors into the per-query buffer;
//   5. one wavefront per query ranks its survivors and writes the output row.
#pragma clang fp contract(off)

#include "tail.hpp"

namespace knn {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = kBlock * 16;  // points per block
constexpr int TNB = 64;
constexpr int kTailShift = 50;

enum Mode : int { kBin = 0, kRefine = 1, kKey = 2 };

__device__ __forceinline__ int tbin(double d2, int64_t top) {
  const int64_t k = (int64_t)((uint64_t)__double_as_longlong(d2) >> kTailShift) - top + (TNB - 1);
  return k < 0 ? 0 : (k > TNB - 1 ? TNB - 1 : (int)k);
}

__device__ __forceinline__ double tail_d2(const double* __restrict__ X, int64_t N, int n,
                                          int64_t p, const double* qx) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) {
    double t = __dsub_rn(X[(int64_t)j * N + p], qx[j]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

__device__ __forceinline__ void load_query(const TailArgs& a, int qi, double* qx, int64_t& qid) {
  qid = a.q_ids[qi];
  for (int j = 0; j < a.n; ++j) qx[j] = a.X[(int64_t)j * a.N + qid];
}

__global__ void k_tail_hist(const TailArgs a) {
  __shared__ uint32_t h[TNB];
  const int qi = blockIdx.y;
  if (threadIdx.x < TNB) h[threadIdx.x] = 0;
  __syncthreads();
  double qx[kMaxDims];
  int64_t qid;
  load_query(a, qi, qx, qid);
  const int64_t p0 = (int64_t)blockIdx.x * kChunk;
  const int64_t p1 = p0 + kChunk < a.N ? p0 + kChunk : a.N;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
    if (p == qid) continue;
    atomicAdd(&h[tbin(tail_d2(a.X, a.N, a.n, p, qx), a.top)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < TNB && h[threadIdx.x]) atomicAdd(&a.hist[qi * TNB + threadIdx.x], h[threadIdx.x]);
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

// Per query in refinement: four thresholds splitting [A, B]; written to state.
__global__ void k_tail_split(const TailArgs a) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.A) return;
  TailState& st = a.state[qi];
  if (st.mode != kRefine) return;
  const unsigned __int128 span = st.B - st.A + 1;
  const unsigned __int128 step = span / 4;
  for (int i = 0; i < 4; ++i) {
    if (i == 3)
      st.t[i] = st.B;
    else if (step == 0)
      st.t[i] = (st.A + (unsigned __int128)i < st.B) ? st.A + (unsigned __int128)i : st.B;
    else
      st.t[i] = st.A - 1 + step * (unsigned __int128)(i + 1);
    a.cnt[qi * 4 + i] = 0;
  }
}

__global__ void k_tail_refine_count(const TailArgs a) {
  const int qi = blockIdx.y;
  const TailState& st = a.state[qi];
  if (st.mode != kRefine) return;
  __shared__ uint32_t c4[4];
  if (threadIdx.x < 4) c4[threadIdx.x] = 0;
  __syncthreads();
  double qx[kMaxDims];
  int64_t qid;
  load_query(a, qi, qx, qid);
  const unsigned __int128 A = st.A;
  const unsigned __int128 t0 = st.t[0], t1 = st.t[1], t2 = st.t[2], t3 = st.t[3];
  uint32_t c[4] = {0, 0, 0, 0};
  const int64_t p0 = (int64_t)blockIdx.x * kChunk;
  const int64_t p1 = p0 + kChunk < a.N ? p0 + kChunk : a.N;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
    if (p == qid) continue;
    const double d2 = tail_d2(a.X, a.N, a.n, p, qx);
    const unsigned __int128 k =
        ((unsigned __int128)(uint64_t)__double_as_longlong(d2) << 32) | (uint32_t)p;
    if (k >= A && k <= t3) {
      c[0] += k <= t0;
      c[1] += k <= t1;
      c[2] += k <= t2;
      c[3] += 1;
    }
  }
  for (int i = 0; i < 4; ++i)
    if (c[i]) atomicAdd(&c4[i], c[i]);
  __syncthreads();
  if (threadIdx.x < 4 && c4[threadIdx.x]) atomicAdd(&a.cnt[qi * 4 + threadIdx.x], c4[threadIdx.x]);
}

__global__ void k_tail_refine_update(const TailArgs a) {
  const int qi = blockIdx.x * blockDim.x + threadIdx.x;
  if (qi >= a.A) return;
  TailState& st = a.state[qi];
  if (st.mode != kRefine) return;
  int i = 0;
  while (i < 3 && st.c_lo + (int)a.cnt[qi * 4 + i] < a.K) ++i;
  const int nchi = st.c_lo + (int)a.cnt[qi * 4 + i];
  if (i > 0) {
    const int nclo = st.c_lo + (int)a.cnt[qi * 4 + i - 1];
    st.A = st.t[i - 1] + 1;
    st.c_lo = nclo;
  }
  st.B = st.t[i];
  st.c_hi = nchi;
  if (st.c_hi <= a.cap)
    st.mode = kKey;
  else
    atomicAdd(&a.flag[0], 1);
}

__global__ void k_tail_collect(const TailArgs a) {
  const int qi = blockIdx.y;
  TailState& st = a.state[qi];
  double qx[kMaxDims];
  int64_t qid;
  load_query(a, qi, qx, qid);
  const int mode = st.mode, bsel = st.bsel;
  const unsigned __int128 B = st.B;
  const int64_t p0 = (int64_t)blockIdx.x * kChunk;
  const int64_t p1 = p0 + kChunk < a.N ? p0 + kChunk : a.N;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
    if (p == qid) continue;
    const double d2 = tail_d2(a.X, a.N, a.n, p, qx);
    bool acc;
    if (mode == kBin)
      acc = tbin(d2, a.top) <= bsel;
    else
      acc = (((unsigned __int128)(uint64_t)__double_as_longlong(d2) << 32) | (uint32_t)p) <= B;
    if (acc) {
      const int slot = atomicAdd(&st.fill, 1);
      if (slot < a.cap) {
        a.buf_d[(int64_t)qi * a.cap + slot] = d2;
        a.buf_i[(int64_t)qi * a.cap + slot] = (int32_t)p;
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
  return (size_t)A * (sizeof(TailState) + TNB * 4 + 16 + (size_t)cap * 12) + 256;
}

int tail_run(TailArgs a, char* scratch, hipStream_t s) {
  // carve the scratch: state, hist, cnt, flag, buffers
  char* p = scratch;
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~size_t(255);
    return r;
  };
  a.state = reinterpret_cast<TailState*>(take((size_t)a.A * sizeof(TailState)));
  a.hist = reinterpret_cast<uint32_t*>(take((size_t)a.A * TNB * 4));
  a.cnt = reinterpret_cast<uint32_t*>(take((size_t)a.A * 16));
  a.flag = reinterpret_cast<int32_t*>(take(16));
  a.buf_d = reinterpret_cast<double*>(take((size_t)a.A * a.cap * 8));
  a.buf_i = reinterpret_cast<int32_t*>(take((size_t)a.A * a.cap * 4));
  KNN_HIP(hipMemsetAsync(a.hist, 0, (size_t)a.A * TNB * 4, s));
  const dim3 grid((unsigned)ceil_div(a.N, kChunk), (unsigned)a.A);
  k_tail_hist<<<grid, kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  const int sb = (int)ceil_div(a.A, kBlock);
  KNN_HIP(hipMemsetAsync(a.flag, 0, 16, s));
  k_tail_select<<<sb, kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  int32_t nref = 0;
  KNN_HIP(hipMemcpyAsync(&nref, a.flag, 4, hipMemcpyDeviceToHost, s));
  KNN_HIP(hipStreamSynchronize(s));
  int rounds = 0;
  while (nref > 0) {
    k_tail_split<<<sb, kBlock, 0, s>>>(a);
    KNN_LAUNCHED();
    k_tail_refine_count<<<grid, kBlock, 0, s>>>(a);
    KNN_LAUNCHED();
    KNN_HIP(hipMemsetAsync(a.flag, 0, 4, s));
    k_tail_refine_update<<<sb, kBlock, 0, s>>>(a);
    KNN_LAUNCHED();
    KNN_HIP(hipMemcpyAsync(&nref, a.flag, 4, hipMemcpyDeviceToHost, s));
    KNN_HIP(hipStreamSynchronize(s));
    ++rounds;
    KNN_CHECK(rounds < 200, KNN_EINTERNAL, "tail refinement did not converge");
  }
  k_tail_collect<<<grid, kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  k_tail_finish<<<(unsigned)ceil_div(a.A, 4), kBlock, 0, s>>>(a);
  KNN_LAUNCHED();
  return rounds;
}

}  // namespace knn
