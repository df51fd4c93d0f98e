// search.hip -- the grid KNN search kernel (GPUJoinKernel of Alg. 1, with the
// per-query top-K selection done on the device instead of the host filter).
//
// One wavefront takes one work item: G = 64/T consecutive active queries (in
// cell order), T lanes per query (the paper's t threads per point, Sec. 4.7).
// For each query:
//   1. Candidates are the points of the 3^n adjacent cells, stored as the
//      non-empty ones of 3^(n-1) contiguous row segments of the cell-sorted
//      SoA coordinates.  Each pass copies the segments it needs into an LDS
//      list (segments provably beyond the pass's distance limit are left
//      out), and the T lanes walk the list as one flattened array, so lane
//      utilisation does not depend on the segment lengths.
//   2. Count pass: every candidate's squared distance (summed left to right,
//      every operation rounded) goes through a monotone bin function into a
//      per-query LDS histogram of NB log-spaced bins (read off the exponent
//      and the top mantissa bits of d^2) ending at r^2, where r
//      is the radius that the scanned cells provably cover.  Fewer than K
//      candidates within r^2 means the K nearest cannot be proven from these
//      cells: the query fails and is re-queued for a larger cell side (Alg. 1,
//      findFailedPnts / addFailuresToWorkQueue).
//   3. The first bin whose cumulative count reaches K selects the survivors
//      (every candidate whose bin is not above it).  Since the bin function is
//      monotone in d^2, the survivors are exactly the candidates below some
//      squared distance, so they contain the K nearest.  If that bin would
//      overflow the per-query buffer (cap), an exact bisection on the key
//      (d^2, id) narrows it first (32-way histogram rounds in key space).
//   4. Collect pass: survivors (d^2, id) go to the per-query LDS buffer,
//      bucketed by bin (the histogram, turned into prefix offsets, serves as
//      the bucket cursors: a counting sort).
//   5. Rank pass: a survivor's rank is its bucket's start plus the bucket
//      mates before it in (d^2, id) order; ranks below K go to the output row.
//
// Exactness of the success test: a point outside the scanned cells differs
// from the query by at least 1 + m cell coordinates in some dimension
// (m = distance of the query to its own cell's nearest face, in cells), which
// in coordinates is at least (1 + m)/inv_w minus rounding; r^2 is that
// radius shrunk by a margin that covers every rounding of the cell
// coordinates and of the squared distance.  So every unscanned point has a
// computed d^2 > r^2 and cannot precede a survivor.
#pragma clang fp contract(off)

#include <map>
#include <mutex>
#include <tuple>

#include "kernels.hpp"

namespace knn {

namespace {

// Count-pass bins: NB log-spaced bins of d^2 below the covered radius.  The
// range has to reach the K-th distance of dense cells, which lies far below
// the covered radius; the resolution has to keep the selected bin within the
// per-query buffer (an overflow is resolved exactly by refinement rounds, but
// costs passes).  Around the K-th neighbour a bin's population grows like
// (bin ratio)^(n/2), while a density contrast c moves the K-th distance by
// c^(1/n): so 2-3 dimensions get 4 bins per octave over 16 octaves
// (exponent + 2 mantissa bits), 4-6 dimensions 8 per octave over 8.
constexpr int NB = 64;
template <int DIM>
struct BinShift {
  static constexpr int v = DIM <= 3 ? 50 : 49;
};
constexpr int NB2 = 32;        // bins of one exact-bisection round
constexpr int kLog2NB2 = 5;
// Candidates per lane in flight in the count/collect walks and the waves per
// SIMD the register budget is set for (measured on MI355X with point-major
// coordinates: 2-4 dimensions are best at 4 in flight with 4 waves per SIMD;
// 5-6 dimensions at 2 in flight, 8 % faster than 4, with 2-4 waves alike).
template <int DIM>
struct Unroll {
  static constexpr int v = DIM <= 4 ? 4 : 2;
};
template <int DIM>
struct WavesPerEu {
  static constexpr int v = DIM <= 4 ? 4 : 2;
};
constexpr int kFailBuf = 64;   // failed ids buffered per wavefront before one global append

template <int D>
struct Pow3 {
  static constexpr int v = 3 * Pow3<D - 1>::v;
};
template <>
struct Pow3<0> {
  static constexpr int v = 1;
};

// Coordinates of point p of the point-major sorted array: S = point_stride
// doubles per point, read as S/2 16-byte loads (one address for them all).
// OFF32 (8 S N < 2^32): the byte offset fits 32 bits, so the loads take the
// form scalar base + 32-bit vector offset.
template <int DIM, bool OFF32>
__device__ __forceinline__ void load_point(const double* __restrict__ Xs, uint32_t p,
                                           double (&x)[DIM]) {
  constexpr int S = point_stride(DIM);
  const double2* src =
      OFF32 ? reinterpret_cast<const double2*>(reinterpret_cast<const char*>(Xs) +
                                               p * (uint32_t)(S * sizeof(double)))
            : reinterpret_cast<const double2*>(Xs + (size_t)p * S);
#pragma unroll
  for (int h = 0; h < S / 2; ++h) {
    const double2 t = src[h];
    x[2 * h] = t.x;
    if (2 * h + 1 < DIM) x[2 * h + 1] = t.y;
  }
}

// Coordinates of several candidates, loaded before any is used: a compiler
// barrier between the loads and the arithmetic keeps them all in flight
// (left alone, the scheduler waits on the first candidate's loads one by one).
template <int DIM, bool OFF32, int U>
__device__ __forceinline__ void sq_dist_batch(const double* __restrict__ Xs,
                                              const uint32_t (&p)[U], const double (&q)[DIM],
                                              double (&d2)[U]) {
  double x[U][DIM];
#pragma unroll
  for (int u = 0; u < U; ++u) load_point<DIM, OFF32>(Xs, p[u], x[u]);
  asm volatile("" ::: "memory");
#pragma unroll
  for (int u = 0; u < U; ++u) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double t = __dsub_rn(x[u][j], q[j]);
      s = __dadd_rn(s, __dmul_rn(t, t));
    }
    d2[u] = s;
  }
}

template <int DIM, bool OFF32>
__device__ __forceinline__ double sq_dist(const double* __restrict__ Xs, uint32_t p,
                                          const double (&q)[DIM]) {
  double x[DIM];
  load_point<DIM, OFF32>(Xs, p, x);
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double t = __dsub_rn(x[j], q[j]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

// Monotone bin of a squared distance: 0..NB-1 for d2 <= thr, NB above it.
// top = (bit pattern of the reference top) >> kBinShift, top0 = top - (NB-1);
// the bit pattern of a non-negative double is monotone in its value, so the
// bin is monotone in d2.  Only the high word is needed (kBinShift >= 32).
template <int DIM>
__device__ __forceinline__ int bin_clamped(double d2, int top0) {
  constexpr int kBinShift = BinShift<DIM>::v;
  const int k = (int)((uint32_t)__double2hiint(d2) >> (kBinShift - 32)) - top0;
  // clamp to [0, NB - 1] in one instruction (the compiler splits min(max())
  // into three here)
  int b;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(b) : "v"(k), "i"(NB - 1));
  return b;
}
template <int DIM>
__device__ __forceinline__ int bin_of(double d2, double thr, int top0) {
  return d2 > thr ? NB : bin_clamped<DIM>(d2, top0);
}

// top0 of a reference squared distance, opaque to the optimizer (which would
// otherwise fold the subtraction back into every bin computation)
template <int DIM>
__device__ __forceinline__ int bin_top0(double ref) {
  int t = (int)((uint64_t)__double_as_longlong(ref) >> BinShift<DIM>::v) - (NB - 1);
  asm("" : "+v"(t));
  return t;
}

// Upper limit of the squared distances in bins 0..b (for pruning the passes
// that only need those bins): below the next bin edge, and never above thr.
template <int DIM>
__device__ __forceinline__ double bins_limit(int b, double thr, int top0) {
  constexpr int kBinShift = BinShift<DIM>::v;
  const int e = top0 + b + 1;  // bit pattern >> kBinShift of the next edge
  if (b >= NB - 1 || e <= 0 || e >= (0x7FF0 >> (kBinShift - 48))) return thr;
  const double edge = __longlong_as_double((long long)((uint64_t)e << kBinShift));
  return fmin(edge, thr);
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int T>
__device__ __forceinline__ int group_incl_scan(int v, int l) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) {
    int u = __shfl_up(v, o, T);
    if (l >= o) v += u;
  }
  return v;
}
template <int T>
__device__ __forceinline__ int group_sum_int(int v) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int T>
__device__ __forceinline__ int group_min_int(int v) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
template <int T>
__device__ __forceinline__ int group_max_int(int v) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
template <int T>
__device__ __forceinline__ double group_min(double v) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
template <int T>
__device__ __forceinline__ double group_max(double v) {
#pragma unroll
  for (int o = 1; o < T; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int bitlen128(unsigned __int128 v) {
  const uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
  return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}

// Per-query candidate list in LDS: the non-empty row segments that a pass
// needs, compacted, as (sorted position minus virtual position, running end in
// virtual candidate numbering).  A segment (or its first or last cell along the last
// dimension) is left out when a conservative lower bound of the squared
// distance from the query to any of its points exceeds the pass's limit (all
// its candidates would be beyond it).  The bound uses the query's distances
// to its own cell's faces: a neighbour at offset +1 in dimension j
// is at least (1 - fr_j - mg) w away, at offset -1 at least (fr_j - mg) w,
// where fr_j is the query's exact fractional cell coordinate and mg bounds
// the rounding of both cell coordinates in cell units; the final factor
// (1 - 2^-40) covers the rounding of the bound and of the computed d2.
constexpr double kBoundShrink = 1.0 - 0x1p-40;

template <int DIM>
__device__ __forceinline__ double seg_bound(int slot, const double (&flo)[DIM],
                                            const double (&fhi)[DIM]) {
  double s = 0.0;
  int rr = slot;
#pragma unroll
  for (int j = DIM - 2; j >= 0; --j) {
    const int o = rr % 3;
    rr /= 3;
    const double d = o == 0 ? flo[j] : (o == 2 ? fhi[j] : 0.0);
    s += d * d;
  }
  return s;
}

// Builds the list of one query (its T lanes call it together; nr_w is the
// wavefront's maximum segment count, so every lane takes the same trips and
// the group exchanges stay converged).  Returns the list's candidate count.
template <int DIM, int T>
__device__ __forceinline__ uint32_t build_list(const uint32_t* __restrict__ rg,
                                               const uint8_t* __restrict__ rs, int nr, int nr_w,
                                               bool prune, double lim, const double (&qx)[DIM],
                                               const SearchArgs& a, int l, uint32_t* seg_of,
                                               uint32_t* seg_ve, bool shared) {
  // face distances (recomputed here rather than kept live through the passes)
  double flo[DIM], fhi[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    const double u = __dmul_rn(__dsub_rn(qx[j], a.lo[j]), a.inv_w);
    const double fr = u - floor(u);  // exact
    flo[j] = fmax(fr - a.margin, 0.0) * a.w;
    fhi[j] = fmax((1.0 - fr) - a.margin, 0.0) * a.w;
  }
  // the last dimension: the segment's lower / upper cells are a face away
  const double dlo = flo[DIM - 1] * flo[DIM - 1], dhi = fhi[DIM - 1] * fhi[DIM - 1];
  uint32_t total = 0, cnt = 0;
  for (int i0 = 0; i0 < nr_w; i0 += T) {
    const int i = i0 + l;
    uint32_t st = 0, len = 0;
    if (i < nr) {
      const uint4 r4 = reinterpret_cast<const uint4*>(rg)[i];  // start, mid0, mid1, end
      if (!prune) {
        st = r4.x;
        len = r4.w - r4.x;
      } else {
        // the middle cells are never farther than the outer ones, so the
        // kept part of a segment is contiguous
        const double b0 = seg_bound<DIM>(rs[i], flo, fhi);
        if (b0 * kBoundShrink <= lim) {
          st = (b0 + dlo) * kBoundShrink <= lim ? r4.x : r4.y;
          const uint32_t en = (b0 + dhi) * kBoundShrink <= lim ? r4.w : r4.z;
          len = en - st;
        }
      }
    }
    if (shared) {
      // every group of the wavefront has the same cell: keep the union of
      // their ranges, so all groups walk one list and each load serves them all
      uint32_t lo = len ? st : 0xFFFFFFFFu, hi = len ? st + len : 0u;
#pragma unroll
      for (int o = T; o < 64; o <<= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
      }
      st = lo;
      len = hi > lo ? hi - lo : 0u;
    }
    const uint32_t keep = len > 0 ? 1u : 0u;
    uint32_t ik = keep, il = len;
#pragma unroll
    for (int o = 1; o < T; o <<= 1) {
      const uint32_t uk = __shfl_up(ik, o, T);
      const uint32_t ul = __shfl_up(il, o, T);
      if (l >= o) {
        ik += uk;
        il += ul;
      }
    }
    if (keep) {
      // offset from virtual to sorted position (mod 2^32): the segment's
      // virtual start is total + il - len
      seg_of[cnt + ik - 1] = st - (total + il - len);
      seg_ve[cnt + ik - 1] = total + il;
    }
    cnt += __shfl(ik, T - 1, T);
    total += __shfl(il, T - 1, T);
  }
  if (l == 0) {  // sentinel: ends every walk (its offset is never used in a valid list)
    seg_of[cnt] = 0;
    seg_ve[cnt] = 0xFFFFFFFFu;
  }
  return total;
}

// Walk over a list: virtual candidate v (non-decreasing from call to call,
// below the list's count) -> sorted position.  Every list ends with a
// sentinel entry whose end is 0xFFFFFFFF, so a walk can never go past it,
// and positions are clamped below N: a list inconsistent with its count
// cannot make the walk loop or read out of bounds (the refinement rounds
// detect the inconsistent counts and report them).
struct LWalk {
  const uint32_t* of;
  const uint32_t* ve;
  int r;
  uint32_t vend, off, last;
  __device__ __forceinline__ void init(const uint32_t* of_, const uint32_t* ve_, uint32_t nlast) {
    of = of_;
    ve = ve_;
    r = 0;
    vend = ve[0];
    off = of[0];
    last = nlast;
  }
  __device__ __forceinline__ uint32_t pos(uint32_t v) {
    while (v >= vend) {
      ++r;
      vend = ve[r];
      off = of[r];
    }
    return min(off + v, last);
  }
};

// Positions of the batch of virtual candidates v, v + T, ..., v + (U-1) T of
// a walk; slots at or past the list's count C get `pad`.  kWhole: the caller
// knows that the whole batch lies inside the list.
template <int T, int U, bool kWhole>
__device__ __forceinline__ void batch_pos(LWalk& cs, uint32_t v, uint32_t C, uint32_t pad,
                                          uint32_t (&p)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t vv = v + (uint32_t)(u * T);
    p[u] = (kWhole || vv < C) ? cs.pos(vv) : pad;
  }
}

// Appends the wavefront's buffered failed ids to the global failure list.
__device__ __forceinline__ void flush_failures(const SearchArgs& a, const int32_t* fbuf, int nfail,
                                               int lane) {
  int base = 0;
  if (lane == 0) base = atomicAdd(a.fail_count, nfail);
  base = __shfl(base, 0, 64);
  for (int i = lane; i < nfail; i += 64) a.fail_list[base + i] = fbuf[i];
  wave_fence();
}

// ZL: a Z-order level, whose cells list the 3^n cells of their block one by
// one (else the 3^(n-1) row segments).
template <int DIM, int T, bool OFF32, bool ZL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WavesPerEu<DIM>::v)))
k_search(const SearchArgs a) {
  constexpr int G = 64 / T;  // queries per wave
  constexpr int R = ZL ? Pow3<DIM>::v : Pow3<DIM - 1>::v;
  constexpr int P = NB / T;  // count bins owned by each lane of a group
  constexpr int kUnroll = Unroll<DIM>::v;
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int g = lane / T;
  const int l = lane % T;
  const int cap = a.cap;
  const int K = a.K;
  const int64_t N = a.N;
  const uint32_t nlast = (uint32_t)(N - 1);
  const int32_t* __restrict__ perm = a.perm;
  const double* __restrict__ Xs = a.Xs;  // point-major sorted coordinates

  // per-wave LDS: survivors d2 [cap][G], survivor ids [cap][G], histogram
  // [NB][G], failure buffer, candidate lists [G][R] (starts, ends); the
  // refinement histogram [NB2][G] reuses the d2 area (it is free before the
  // collect, and cap >= NB2/2 + 1).
  int32_t* bi_base = reinterpret_cast<int32_t*>(smem + (size_t)nwaves * cap * G);
  uint32_t* hist_base = reinterpret_cast<uint32_t*>(bi_base + (size_t)nwaves * cap * G);
  int32_t* fbuf_base = reinterpret_cast<int32_t*>(hist_base + (size_t)nwaves * (NB + 1) * G);
  uint32_t* seg_base = reinterpret_cast<uint32_t*>(fbuf_base + (size_t)nwaves * kFailBuf);
  double* bd = smem + (size_t)wave * cap * G;
  int32_t* bi = bi_base + (size_t)wave * cap * G;
  uint32_t* hist = hist_base + (size_t)wave * (NB + 1) * G;
  uint32_t* hist2 = reinterpret_cast<uint32_t*>(bd);
  int32_t* fbuf = fbuf_base + (size_t)wave * kFailBuf;
  uint32_t* seg_of = seg_base + (size_t)wave * 2 * (R + 1) * G + (size_t)g * (R + 1);
  uint32_t* seg_ve = seg_of + (size_t)(R + 1) * G;
  // speculative survivors of group g: slot k at spos[k * G + g] (SC slots),
  // their count in hist[NB * G + g]
  const int SC = a.spec_slots;
  uint32_t* spos = seg_base + (size_t)nwaves * 2 * (R + 1) * G + (size_t)wave * SC * G;
  // Speculation: the K-th squared distance of a query is predicted from the
  // point density of its cell's 3^n block (C points in (3w)^n): a ball
  // holding K points there has d^n = K (3w)^n / (C V_n), so
  // d^2 = spec_coef * C^(-2/n), spec_coef including a safety factor.  The
  // count pass keeps the positions of the candidates within that limit; if
  // they turn out to hold at least K candidates (so all K nearest) without
  // overflowing, the survivors are bucketed from them and the collect pass
  // over the whole list is skipped.
  int spec_held = 0;  // wavefront total (lane 0), added to a.spec_count at the end

  const uint64_t lane_lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));

  // Persistent schedule: one work queue per XCD.  Workgroups are dispatched
  // round-robin over the 8 XCDs, so blockIdx % 8 names the XCD; queue x holds
  // a contiguous (in cell order, so spatially local) eighth of the items,
  // densest class first, which keeps each XCD's L2 on one region of the grid.
  // An exhausted queue sends the wavefront on to the next XCD's queue.
  // Pops claim `grain` consecutive items at a time, so the queue heads see one
  // atomic per grain, not per item.
  int qx = (int)(blockIdx.x % kXcds);
  int tried = 0;
  int64_t cur = 0, end = 0;  // claimed order positions [cur, end)
  bool first = true;
  // Failed query ids are buffered per wavefront in LDS and appended to the
  // global list kFailBuf at a time (one atomic per flush).
  int nfail = 0;
  for (;;) {
    int64_t item;
    if (a.persistent) {
      while (cur >= end && tried < kXcds) {
        int v = 0;
        if (lane == 0) {
          // a plain load first: drained queues cost no atomic
          int32_t* hp = a.head + qx * kLineInts;
          v = __hip_atomic_load(hp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (a.qbeg[qx] + v < a.qbeg[qx + 1]) v = atomicAdd(hp, a.grain);
        }
        v = __shfl(v, 0, 64);
        const int64_t b = a.qbeg[qx] + v;
        if (b < a.qbeg[qx + 1]) {
          cur = b;
          end = min(b + (int64_t)a.grain, a.qbeg[qx + 1]);
        } else {
          qx = (qx + 1) % kXcds;
          ++tried;
        }
      }
      if (cur >= end) break;
      item = cur++;
    } else {
      if (!first) break;
      item = a.item_base + (int64_t)blockIdx.x * nwaves + wave;
      if (item >= a.n_items) break;
    }
    first = false;
    const int64_t it = a.order ? (int64_t)a.order[item] : item;
    const int64_t slot = it * G + g;
    const bool in = slot < a.n_active;
    const int64_t q = in ? (a.active ? (int64_t)a.active[slot] : slot) : 0;
    const uint32_t q32 = (uint32_t)q;

    // ---- query point, covered radius, face distances ------------------------
    double qx[DIM];
    load_point<DIM, false>(Xs, (uint32_t)q, qx);
    const uint32_t cell = a.cell_of[q];
    const uint32_t* rg = a.ranges + (size_t)cell * R * 4;
    const uint8_t* rs = a.rslot + (size_t)cell * R;
    const uint32_t Cq = in ? a.cand[cell] : 0u;
    // heavy queries are handled by k_search_heavy
    const bool valid = in && (a.heavy_min == 0 || Cq < a.heavy_min);
    // K-th distance prediction from the 3^n block's density (C^(-2/n))
    const double dpred =
        SC > 0 && Cq > 0 ? a.spec_coef * (double)powf((float)Cq, -2.0f / DIM) : -1.0;
    const int nr = valid ? (int)a.nrng[cell] : 0;
    double mfrac = 0.5;
    bool full = true;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      double u = __dmul_rn(__dsub_rn(qx[j], a.lo[j]), a.inv_w);
      double fl = floor(u);
      double fr = u - fl;  // exact
      mfrac = fmin(mfrac, fmin(fr, 1.0 - fr));
      int64_t c = (int64_t)fl;
      if (c > 1 || c < a.g[j] - 2) full = false;
    }
    double thr, ref;
    if (full) {
      // the scanned cells hold every point: all candidates count; the bins end
      // at the squared diagonal of the 3^n block
      thr = INFINITY;
      ref = 9.0 * DIM * a.w * a.w;
    } else {
      double base = (1.0 + mfrac) * a.w;
      double r = base * (1.0 - a.margin);
      thr = r * r;
      ref = thr;
    }
    const int top0 = bin_top0<DIM>(ref);
    int nr_w = nr;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) nr_w = max(nr_w, __shfl_xor(nr_w, o, 64));
    // one candidate list for the whole wavefront when all its queries share a
    // cell (lists of queries of one cell differ only by pruning)
    bool shared = false;
    if (a.share_lists && G > 1) {
      uint32_t cmin = valid ? cell : 0xFFFFFFFFu, cmax = valid ? cell : 0u;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        cmin = min(cmin, (uint32_t)__shfl_xor((int)cmin, o, 64));
        cmax = max(cmax, (uint32_t)__shfl_xor((int)cmax, o, 64));
      }
      shared = cmin == cmax;
    }

    // ---- count pass over the segments that can hold a point within thr -----
    uint32_t C =
        build_list<DIM, T>(rg, rs, nr, nr_w, !full, thr, qx, a, l, seg_of, seg_ve, shared);
    for (int b = l; b <= NB; b += T) hist[b * G + g] = 0;
    wave_fence();
    {
      LWalk cs;
      cs.init(seg_of, seg_ve, nlast);
      // positions first, then all coordinate loads in flight together
      auto count = [&](const uint32_t (&p)[kUnroll]) {
        double d2[kUnroll];
        sq_dist_batch<DIM, OFF32, kUnroll>(Xs, p, qx, d2);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (!(d2[u] > thr)) atomicAdd(&hist[bin_clamped<DIM>(d2[u], top0) * G + g], 1u);
          if (d2[u] <= dpred && p[u] != q32) {
            const uint32_t k = atomicAdd(&hist[NB * G + g], 1u);
            if ((int)k < SC) spos[k * G + g] = p[u];
          }
        }
      };
      uint32_t v = l;
      for (; v + (kUnroll - 1) * T < C; v += T * kUnroll) {
        uint32_t p[kUnroll];
        batch_pos<T, kUnroll, true>(cs, v, C, q32, p);
        count(p);
      }
      if (v < C) {
        uint32_t p[kUnroll];
        batch_pos<T, kUnroll, false>(cs, v, C, q32, p);
        count(p);
      }
    }
    // The walk counted the query itself (its own cell is always in the list
    // of a self-join) and every slot past the list's end (given the query's
    // position): all at distance 0, in bin bin_of(0).  Each lane takes back
    // its own padding slots, lane 0 also the query (external queries are in
    // no list).
    if (valid) {
      const uint32_t it = l < (int)C ? (C - (uint32_t)l + T * kUnroll - 1) / (T * kUnroll) : 0u;
      const uint32_t real = l < (int)C ? (C - (uint32_t)l + T - 1) / T : 0u;
      const uint32_t back = it * kUnroll - real + (l == 0 && a.self_in_list ? 1u : 0u);
      if (back) atomicSub(&hist[bin_of<DIM>(0.0, thr, top0) * G + g], back);
    }
    wave_fence();

    // ---- selection ---------------------------------------------------------
    // Lane l of the group owns bins [l*P, (l+1)*P).  A group scan of the
    // per-lane sums gives every bin's prefix; the first bin whose cumulative
    // count reaches K is the selected bin, and the histogram is rewritten in
    // place as exclusive prefixes (the bucket cursors of the collect).
    int bsel = NB, c_lo = 0, c_hi = 0;
    {
      uint32_t* hb = hist + (size_t)(l * P) * G + g;
      int local = 0;
      for (int i = 0; i < P; ++i) local += (int)hb[i * G];
      const int incl = group_incl_scan<T>(local, l);
      int mb = NB, mlo = 0, mhi = 0;
      int cum = incl - local;
      for (int i = 0; i < P; ++i) {
        const int h = (int)hb[i * G];
        if (mb == NB && cum + h >= K) {
          mb = l * P + i;
          mlo = cum;
          mhi = cum + h;
        }
        hb[i * G] = (uint32_t)cum;
        cum += h;
      }
      bsel = group_min_int<T>(mb);
      c_lo = group_max_int<T>(mb == bsel ? mlo : 0);
      c_hi = group_max_int<T>(mb == bsel ? mhi : 0);
    }
    const bool fail = valid && bsel == NB;
    const bool ok = valid && bsel < NB;

    // ---- failures: re-queue (buffered per wavefront) ------------------------------
    {
      const bool lf = fail && l == 0;
      const uint64_t fm = __ballot(lf);
      if (fm) {
        const int nf = (int)__popcll(fm);
        if (nfail + nf > kFailBuf) {
          flush_failures(a, fbuf, nfail, lane);
          nfail = 0;
        }
        if (lf) fbuf[nfail + (int)__popcll(fm & lane_lt)] = a.fail_pos ? (int32_t)q : perm[q];
        nfail += nf;
        wave_fence();
      }
    }

    // ---- speculation outcome ------------------------------------------------
    // The kept candidates (d2 <= dpred) number sn.  sn >= K puts the K-th
    // smallest d2 at or below dpred, so they include every candidate of the
    // bins below bsel and every candidate of bin bsel that can rank below K
    // (any other has d2 > dpred, so K candidates precede it).
    const int sn = (int)hist[NB * G + g];
    const bool spec = ok && c_hi <= cap && sn >= K && sn <= SC;
    {
      const int held = (int)__popcll(__ballot(spec && l == 0));
      if (lane == 0) spec_held += held;
    }

    // ---- list for the remaining passes: only bins up to the selected one ----
    const double lim2 = ok ? bins_limit<DIM>(bsel, thr, top0) : 0.0;
    C = build_list<DIM, T>(rg, rs, ok && !spec ? nr : 0, nr_w, true, lim2, qx, a, l, seg_of,
                           seg_ve, shared);
    wave_fence();

    // ---- exact refinement when the selected bin overflows the buffer -------
    // Keys are (d2 bits, id) as 96-bit integers; [A, B] is an inclusive key
    // interval with c_lo keys below A and c_hi keys up to B, c_lo < K <= c_hi.
    // Each round counts the keys of [A, B] into NB2 equal key sub-ranges and
    // keeps the first one where the count reaches K: the interval shrinks at
    // least NB2/2-fold, and a single-key interval holds at most one candidate.
    bool refine = ok && c_hi > cap;
    const bool refined = refine;
    unsigned __int128 B = 0;  // final threshold when refined
    if (__ballot(refine)) {
      // exact value bounds of the selected bin
      double dmin = INFINITY, dmax = -INFINITY;
      {
        LWalk cs;
        cs.init(seg_of, seg_ve, nlast);
        const uint32_t Cr = refine ? C : 0u;
        for (uint32_t v = l; v < Cr; v += T) {
          const uint32_t p = cs.pos(v);
          if (p != q32) {
            const double d2 = sq_dist<DIM, OFF32>(Xs, p, qx);
            if (bin_of<DIM>(d2, thr, top0) == bsel) {
              dmin = fmin(dmin, d2);
              dmax = fmax(dmax, d2);
            }
          }
        }
        }
      dmin = group_min<T>(dmin);
      dmax = group_max<T>(dmax);
      unsigned __int128 A = 0;
      if (refine) {
        A = (unsigned __int128)(uint64_t)__double_as_longlong(dmin) << 32;
        B = ((unsigned __int128)(uint64_t)__double_as_longlong(dmax) << 32) | 0xFFFFFFFFu;
      }
      int rounds = 0;
      while (__ballot(refine)) {
        ++rounds;
        int sh = refine ? bitlen128(B - A) - kLog2NB2 : 0;
        if (sh < 0) sh = 0;
        for (int b = l; b < NB2; b += T) hist2[b * G + g] = 0;
        wave_fence();
        {
          const uint64_t ahi = (uint64_t)(A >> 32), bhi = (uint64_t)(B >> 32);
          LWalk cs;
          cs.init(seg_of, seg_ve, nlast);
          const uint32_t Cr = refine ? C : 0u;
          for (uint32_t v = l; v < Cr; v += T) {
            const uint32_t p = cs.pos(v);
            if (p != q32) {
              const double d2 = sq_dist<DIM, OFF32>(Xs, p, qx);
              const uint64_t kh = (uint64_t)__double_as_longlong(d2);
              if (kh >= ahi && kh <= bhi) {
                const unsigned __int128 k = ((unsigned __int128)kh << 32) | (uint32_t)perm[p];
                if (k >= A && k <= B) atomicAdd(&hist2[(int)((k - A) >> sh) * G + g], 1u);
              }
            }
          }
            }
        wave_fence();
        if (refine) {
          int cum = c_lo;
          bool found = false;
          for (int b = 0; b < NB2; ++b) {
            const int h = (int)hist2[b * G + g];
            if (cum + h >= K) {
              const unsigned __int128 nA = A + ((unsigned __int128)b << sh);
              const unsigned __int128 nB = nA + (((unsigned __int128)1 << sh) - 1);
              A = nA;
              B = nB < B ? nB : B;
              c_lo = cum;
              c_hi = cum + h;
              found = true;
              break;
            }
            cum += h;
          }
          // The counts of [A, B] always reach K, and a single-key interval
          // holds at most one candidate (so c_hi <= K there); otherwise the
          // passes disagreed: stop and report instead of looping.
          if (c_hi <= cap) {
            refine = false;
          } else if (!found || A == B) {
            refine = false;
            if (l == 0) atomicAdd(a.walk_error, 1);
          }
        }
        wave_fence();
      }
      if (l == 0 && refined && a.refine_count) atomicAdd(a.refine_count, rounds);
    }
    const double th_d = __longlong_as_double((long long)(uint64_t)(B >> 32));
    const uint32_t th_id = (uint32_t)(B & 0xFFFFFFFFu);

    // ---- collect pass: survivors bucketed by bin (counting sort) --------------
    wave_fence();
    {
      LWalk cs;
      cs.init(seg_of, seg_ve, nlast);
      auto collect = [&](const uint32_t (&pp)[kUnroll]) {
        double dd[kUnroll];
        sq_dist_batch<DIM, OFF32, kUnroll>(Xs, pp, qx, dd);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t p = pp[u];
          const double d2 = dd[u];
          const int b = bin_of<DIM>(d2, thr, top0);
          bool acc;
          if (refined)
            acc = d2 < th_d || (d2 == th_d && (th_id == 0xFFFFFFFFu || (uint32_t)perm[p] <= th_id));
          else
            acc = b <= bsel;
          // only queries that selected a bin collect: a failed or empty slot
          // walking a shared list has bsel == NB, and bin NB is not a bucket
          // (a speculating query collects from its kept candidates below)
          if (ok && !spec && p != q32 && acc) {
            const uint32_t s = atomicAdd(&hist[b * G + g], 1u);
            if ((int)s < cap) {
              bd[s * G + g] = d2;
              bi[s * G + g] = perm[p];
            }
          }
        }
      };
      uint32_t v = l;
      for (; v + (kUnroll - 1) * T < C; v += T * kUnroll) {
        uint32_t pp[kUnroll];
        batch_pos<T, kUnroll, true>(cs, v, C, q32, pp);
        collect(pp);
      }
      if (v < C) {
        uint32_t pp[kUnroll];
        batch_pos<T, kUnroll, false>(cs, v, C, q32, pp);
        collect(pp);
      }
    }
    if (spec) {
      // the kept candidates of bins up to bsel, into their buckets
      for (int k = l; k < sn; k += T) {
        const uint32_t p = spos[k * G + g];
        const double d2 = sq_dist<DIM, OFF32>(Xs, p, qx);
        const int b = bin_of<DIM>(d2, thr, top0);
        if (b <= bsel) {
          const uint32_t s = atomicAdd(&hist[b * G + g], 1u);
          if ((int)s < cap) {
            bd[s * G + g] = d2;
            bi[s * G + g] = perm[p];
          }
        }
      }
    }
    wave_fence();

    // ---- rank pass -> output row ------------------------------------------------
    // After the collect, hist[b] is the end of bucket b, and bucket b starts at
    // the end of bucket b-1; a survivor's rank is its bucket start plus the
    // number of bucket mates before it in (d2, id) order.
    const int c = ok ? min((int)hist[bsel * G + g], cap) : 0;
    const int64_t row = ok ? (int64_t)perm[q] : 0;
    for (int a0 = 0; a0 < c; a0 += T) {
      const int ai = a0 + l;
      if (ai < c) {
        const double da = bd[ai * G + g];
        const int32_t ia = bi[ai * G + g];
        const int b = bin_of<DIM>(da, thr, top0);
        const int start = b > 0 ? (int)hist[(b - 1) * G + g] : 0;
        if (start < K) {
          const int end = min((int)hist[b * G + g], cap);
          int rank = start;
          for (int s2 = start; s2 < end; ++s2) {
            const double db = bd[s2 * G + g];
            const int32_t ib = bi[s2 * G + g];
            rank += (db < da || (db == da && ib < ia)) ? 1 : 0;
          }
          if (rank < K) {
            a.out_ids[row * K + rank] = ia;
            a.out_d[row * K + rank] = sqrt(da);
          }
        }
      }
    }
    wave_fence();
  }
  if (nfail > 0) flush_failures(a, fbuf, nfail, lane);
  if (lane == 0 && spec_held > 0 && a.spec_count) atomicAdd(a.spec_count, spec_held);
}

// Deferral filter: a tile is kDeferRounds rounds of 64 consecutive active
// slots per wavefront (coalesced); keep / defer decisions are ballots.  Three
// launches: the decisions (with the skip-ahead flags, pending counts and
// candidate sums) store their ballots and each tile's kept count, a scan of
// the counts, and a pass that compacts the kept slots in order from the
// ballots and appends deferred ids after one atomic per block.
constexpr int kDeferRounds = 8;
constexpr int kDeferTile = 256 * kDeferRounds;
static_assert(kDeferTile >= kLbMinTile, "tile area sized for larger tiles");

// ballots of wavefront w of a tile, round k: keep, then defer
__device__ inline unsigned long long* defer_masks(const DeferArgs& a, int64_t tile, int w, int k) {
  return reinterpret_cast<unsigned long long*>(a.tile_masks) +
         2 * ((tile * 4 + w) * kDeferRounds + k);
}

template <int DIM>
__global__ void __launch_bounds__(256) k_defer_filter(const DeferArgs a) {
  __shared__ uint32_t s_wk[4];
  __shared__ unsigned long long s_sum[4], s_max[4];
  __shared__ uint32_t s_pend[KNN_MAX_LEVELS];  // deferrals per target level (skip-ahead)
  if (a.failed)
    for (int i = threadIdx.x; i < KNN_MAX_LEVELS; i += blockDim.x) s_pend[i] = 0;
  __syncthreads();
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t wbase = tile * kDeferTile + (int64_t)w * 64 * kDeferRounds;
  uint32_t nk = 0;
  unsigned long long csum = 0, cmax = 0;
  const int64_t n_act = a.n_active_dev ? min(a.n_active, (int64_t)*a.n_active_dev) : a.n_active;
  const uint32_t M = a.cell_key ? *a.d_M : 0u;
#pragma unroll
  for (int k = 0; k < kDeferRounds; ++k) {
    const int64_t i = wbase + k * 64 + lane;
    const bool in = i < n_act;
    const int32_t q = in ? (a.active ? a.active[i] : (int32_t)i) : 0;
    bool defer = false;
    uint32_t Cq = 0;
    if (in) {
      double qx[DIM];
      load_point<DIM, false>(a.Xs, (uint32_t)q, qx);
      const uint32_t c = a.cell_of[q];
      if (a.cell_key) {
        // the points of the parent group: the cells next to c in the table
        // whose keys agree above the last DIM bits (at most 2^DIM of them)
        const uint64_t pk = a.cell_key[c] >> DIM;
        uint32_t c0 = c, c1 = c;
        while (c0 > 0 && (a.cell_key[c0 - 1] >> DIM) == pk) --c0;
        while (c1 + 1 < M && (a.cell_key[c1 + 1] >> DIM) == pk) ++c1;
        Cq = a.cell_start[c1 + 1] - a.cell_start[c0];
      } else {
        Cq = a.cand[c];
      }
      // the covered radius of the search kernel
      double mfrac = 0.5;
      bool full = true;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        const double u = __dmul_rn(__dsub_rn(qx[j], a.lo[j]), a.inv_w);
        const double fl = floor(u);
        const double fr = u - fl;
        mfrac = fmin(mfrac, fmin(fr, 1.0 - fr));
        const int64_t c = (int64_t)fl;
        if (c > 1 || c < a.g[j] - 2) full = false;
      }
      const double r = (1.0 + mfrac) * a.w * (1.0 - a.margin);
      const double pd = Cq > 0 ? a.defer_coef * (double)powf((float)Cq, -2.0f / DIM) : 0.0;
      defer = !full && Cq > 0 && pd > r * r;
      if (defer && a.failed) {
        // skip ahead: the first level L' > level with 1.5 w 2^(L' - level)
        // >= sqrt(pd), the smallest side at which the query could succeed
        const float ratio = (float)(sqrt(pd) / (1.5 * a.w));
        int jump = ratio > 2.0f ? (int)ceilf(log2f(ratio)) : 1;
        jump = max(jump, 1);
        const int target = min(a.level + jump, a.top_level);
        a.failed[q] = (uint8_t)target;
        atomicAdd(&s_pend[target], 1u);
      }
    }
    const unsigned long long mk = __ballot(in && !defer);
    const unsigned long long md = __ballot(in && defer);
    nk += (uint32_t)__popcll(mk);
    if (lane == 0) {
      unsigned long long* mm = defer_masks(a, tile, w, k);
      mm[0] = mk;
      mm[1] = md;
    }
    if (in && !defer) {
      csum += Cq;
      cmax = cmax > Cq ? cmax : (unsigned long long)Cq;
    }
  }
  // candidate sum and maximum of the kept queries
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    csum += __shfl_xor(csum, off, 64);
    const unsigned long long m2 = __shfl_xor(cmax, off, 64);
    cmax = cmax > m2 ? cmax : m2;
  }
  if (lane == 0) {
    s_wk[w] = nk;
    s_sum[w] = csum;
    s_max[w] = cmax;
  }
  __syncthreads();
  if (a.failed)
    for (int i = threadIdx.x; i < KNN_MAX_LEVELS; i += blockDim.x)
      if (s_pend[i]) atomicAdd(&a.pending[i], s_pend[i]);
  if (threadIdx.x == 0) {
    unsigned long long ts = 0, tm = 0;
    uint32_t agg = 0;
    for (int i = 0; i < 4; ++i) {
      ts += s_sum[i];
      tm = tm > s_max[i] ? tm : s_max[i];
      agg += s_wk[i];
    }
    a.tile_counts[tile] = agg;
    if (a.cand_sum && ts) atomicAdd(&a.cand_sum[0], ts);
    if (a.cand_sum && tm) atomicMax(&a.cand_sum[1], tm);
  }
}

// The compaction of a tile's decisions: a.tile_counts holds the kept slots
// of all earlier tiles.
__global__ void __launch_bounds__(256) k_defer_write(const DeferArgs a) {
  __shared__ uint32_t s_wk[4], s_wd[4];
  __shared__ uint32_t s_fbase;
  const int64_t tile = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbase = tile * kDeferTile + (int64_t)w * 64 * kDeferRounds;
  unsigned long long mk[kDeferRounds], md[kDeferRounds];
  uint32_t nk = 0, nd = 0;
#pragma unroll
  for (int k = 0; k < kDeferRounds; ++k) {
    const unsigned long long* mm = defer_masks(a, tile, w, k);
    mk[k] = mm[0];
    md[k] = mm[1];
    nk += (uint32_t)__popcll(mk[k]);
    nd += (uint32_t)__popcll(md[k]);
  }
  if (lane == 0) {
    s_wk[w] = nk;
    s_wd[w] = nd;
  }
  __syncthreads();
  uint32_t bk = 0, bd = 0, dagg = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i < w) {
      bk += s_wk[i];
      bd += s_wd[i];
    }
    dagg += s_wd[i];
  }
  if (threadIdx.x == 0)
    s_fbase = dagg && !a.failed ? (uint32_t)atomicAdd(a.fail_count, (int32_t)dagg) : 0u;
  __syncthreads();
  uint32_t o = a.tile_counts[tile] + bk, f = s_fbase + bd;
#pragma unroll
  for (int k = 0; k < kDeferRounds; ++k) {
    const int64_t i = wbase + k * 64 + lane;
    const bool keep = (mk[k] >> lane) & 1ull;
    const bool dfr = ((md[k] >> lane) & 1ull) && !a.failed;
    if (keep || dfr) {
      const int32_t q = a.active ? a.active[i] : (int32_t)i;
      if (keep) a.out_active[o + (uint32_t)__popcll(mk[k] & lt_mask)] = q;
      if (dfr) a.fail_list[f + (uint32_t)__popcll(md[k] & lt_mask)] = a.fail_pos ? q : a.perm[q];
    }
    o += (uint32_t)__popcll(mk[k]);
    f += (uint32_t)__popcll(md[k]);
  }
}

// The same search for one query per workgroup of kHeavyThreads lanes: the
// queries of a level whose candidate count is far above the level's mean
// (next to dense regions after the cell side has grown), which would keep a
// single wavefront busy long after the rest of the level is done.  Same bins,
// lists, selection, refinement and ranking as k_search, with workgroup
// barriers in place of the group's lane exchanges (the lists are built by the
// first wavefront).
template <int DIM, bool ZL>
__global__ void __launch_bounds__(kHeavyThreads) k_search_heavy(const SearchArgs a) {
  constexpr int R = ZL ? Pow3<DIM>::v : Pow3<DIM - 1>::v;
  constexpr int NT = kHeavyThreads;
  constexpr int kUnroll = Unroll<DIM>::v;
  extern __shared__ double smem[];
  __shared__ uint32_t hist[NB];
  __shared__ uint32_t hist2[NB2];
  __shared__ uint32_t seg_of[R + 1], seg_ve[R + 1];
  __shared__ int s_bsel, s_clo, s_chi, s_refine;
  __shared__ uint32_t s_C;
  __shared__ unsigned long long s_dmin, s_dmax;
  __shared__ unsigned __int128 s_A, s_B;
  const int tid = threadIdx.x;
  const int cap = a.cap;
  const int K = a.K;
  const int64_t N = a.N;
  const uint32_t nlast = (uint32_t)(N - 1);
  const int32_t* __restrict__ perm = a.perm;
  const double* __restrict__ Xs = a.Xs;
  double* bd = smem;
  int32_t* bi = reinterpret_cast<int32_t*>(smem + cap);
  const int nh = *a.n_heavy;

  for (int hq = blockIdx.x; hq < nh; hq += gridDim.x) {
    const int64_t q = a.heavy[hq];
    const uint32_t q32 = (uint32_t)q;
    double qx[DIM];
    load_point<DIM, false>(Xs, (uint32_t)q, qx);
    const uint32_t cell = a.cell_of[q];
    const uint32_t* rg = a.ranges + (size_t)cell * R * 4;
    const uint8_t* rs = a.rslot + (size_t)cell * R;
    const int nr = (int)a.nrng[cell];
    double mfrac = 0.5;
    bool full = true;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      double u = __dmul_rn(__dsub_rn(qx[j], a.lo[j]), a.inv_w);
      double fl = floor(u);
      double fr = u - fl;
      mfrac = fmin(mfrac, fmin(fr, 1.0 - fr));
      int64_t c = (int64_t)fl;
      if (c > 1 || c < a.g[j] - 2) full = false;
    }
    double thr, ref;
    if (full) {
      thr = INFINITY;
      ref = 9.0 * DIM * a.w * a.w;
    } else {
      double base = (1.0 + mfrac) * a.w;
      double r = base * (1.0 - a.margin);
      thr = r * r;
      ref = thr;
    }
    const int top0 = bin_top0<DIM>(ref);

    // ---- count pass
    if (tid < 64) {
      const uint32_t C0 =
          build_list<DIM, 64>(rg, rs, nr, nr, !full, thr, qx, a, tid, seg_of, seg_ve, false);
      if (tid == 0) s_C = C0;
      hist[tid] = 0;  // NB == 64
    }
    __syncthreads();
    uint32_t C = s_C;
    {
      LWalk cs;
      cs.init(seg_of, seg_ve, nlast);
      for (uint32_t v = tid; v < C; v += NT * kUnroll) {
        uint32_t p[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t vv = v + (uint32_t)(u * NT);
          p[u] = vv < C ? cs.pos(vv) : q32;
        }
        double d2[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) d2[u] = sq_dist<DIM, false>(Xs, p[u], qx);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int b = bin_of<DIM>(d2[u], thr, top0);
          if (p[u] != q32 && b < NB) atomicAdd(&hist[b], 1u);
        }
      }
    }
    __syncthreads();

    // ---- selection (one lane), histogram -> exclusive prefixes
    if (tid == 0) {
      int cum = 0, bsel = NB, clo = 0, chi = 0;
      for (int b = 0; b < NB; ++b) {
        const int h = (int)hist[b];
        if (bsel == NB && cum + h >= K) {
          bsel = b;
          clo = cum;
          chi = cum + h;
        }
        hist[b] = (uint32_t)cum;
        cum += h;
      }
      s_bsel = bsel;
      s_clo = clo;
      s_chi = chi;
      s_dmin = ~0ull;
      s_dmax = 0ull;
      if (bsel == NB) {
        a.fail_list[atomicAdd(a.fail_count, 1)] = a.fail_pos ? (int32_t)q : perm[q];
        if (a.heavy_fail) atomicAdd(a.heavy_fail, 1);
      }
    }
    __syncthreads();
    const int bsel = s_bsel;
    if (bsel == NB) continue;  // failed: re-queued for a larger cell side

    // ---- list of the remaining passes
    if (tid < 64) {
      const uint32_t C1 = build_list<DIM, 64>(rg, rs, nr, nr, true, bins_limit<DIM>(bsel, thr, top0),
                                              qx, a, tid, seg_of, seg_ve, false);
      if (tid == 0) s_C = C1;
    }
    __syncthreads();
    C = s_C;

    // ---- exact refinement when the selected bin overflows the buffer
    const bool refined = s_chi > cap;
    if (refined) {
      {
        unsigned long long mn = ~0ull, mx = 0ull;
        LWalk cs;
        cs.init(seg_of, seg_ve, nlast);
        for (uint32_t v = tid; v < C; v += NT) {
          const uint32_t p = cs.pos(v);
          if (p != q32) {
            const double d2 = sq_dist<DIM, false>(Xs, p, qx);
            if (bin_of<DIM>(d2, thr, top0) == bsel) {
              const unsigned long long kb = (unsigned long long)__double_as_longlong(d2);
              mn = min(mn, kb);
              mx = max(mx, kb);
            }
          }
        }
        if (mn != ~0ull) atomicMin(&s_dmin, mn);
        if (mx != 0ull) atomicMax(&s_dmax, mx);
        }
      __syncthreads();
      if (tid == 0) {
        s_A = (unsigned __int128)(uint64_t)s_dmin << 32;
        s_B = ((unsigned __int128)(uint64_t)s_dmax << 32) | 0xFFFFFFFFu;
        s_refine = 1;
      }
      __syncthreads();
      int rounds = 0;
      while (s_refine) {
        ++rounds;
        const unsigned __int128 A = s_A, B = s_B;
        int sh = bitlen128(B - A) - kLog2NB2;
        if (sh < 0) sh = 0;
        for (int b = tid; b < NB2; b += NT) hist2[b] = 0;
        __syncthreads();
        {
          const uint64_t ahi = (uint64_t)(A >> 32), bhi = (uint64_t)(B >> 32);
          LWalk cs;
          cs.init(seg_of, seg_ve, nlast);
          for (uint32_t v = tid; v < C; v += NT) {
            const uint32_t p = cs.pos(v);
            if (p != q32) {
              const double d2 = sq_dist<DIM, false>(Xs, p, qx);
              const uint64_t kh = (uint64_t)__double_as_longlong(d2);
              if (kh >= ahi && kh <= bhi) {
                const unsigned __int128 k = ((unsigned __int128)kh << 32) | (uint32_t)perm[p];
                if (k >= A && k <= B) atomicAdd(&hist2[(int)((k - A) >> sh)], 1u);
              }
            }
          }
            }
        __syncthreads();
        if (tid == 0) {
          int cum = s_clo;
          bool found = false;
          for (int b = 0; b < NB2; ++b) {
            const int h = (int)hist2[b];
            if (cum + h >= K) {
              const unsigned __int128 nA = A + ((unsigned __int128)b << sh);
              const unsigned __int128 nB = nA + (((unsigned __int128)1 << sh) - 1);
              s_A = nA;
              s_B = nB < B ? nB : B;
              s_clo = cum;
              s_chi = cum + h;
              found = true;
              break;
            }
            cum += h;
          }
          if (s_chi <= cap) {
            s_refine = 0;
          } else if (!found || s_A == s_B) {
            s_refine = 0;
            atomicAdd(a.walk_error, 1);
          }
        }
        __syncthreads();
      }
      if (tid == 0 && a.refine_count) atomicAdd(a.refine_count, rounds);
    }
    const unsigned __int128 Bf = s_B;
    const double th_d = __longlong_as_double((long long)(uint64_t)(Bf >> 32));
    const uint32_t th_id = (uint32_t)(Bf & 0xFFFFFFFFu);

    // ---- collect pass
    {
      LWalk cs;
      cs.init(seg_of, seg_ve, nlast);
      for (uint32_t v = tid; v < C; v += NT * kUnroll) {
        uint32_t pp[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t vv = v + (uint32_t)(u * NT);
          pp[u] = vv < C ? cs.pos(vv) : q32;
        }
        double dd[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) dd[u] = sq_dist<DIM, false>(Xs, pp[u], qx);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const uint32_t p = pp[u];
          const double d2 = dd[u];
          const int b = bin_of<DIM>(d2, thr, top0);
          bool acc;
          if (refined)
            acc = d2 < th_d || (d2 == th_d && (th_id == 0xFFFFFFFFu || (uint32_t)perm[p] <= th_id));
          else
            acc = b <= bsel;
          if (p != q32 && acc) {
            const uint32_t sidx = atomicAdd(&hist[b], 1u);
            if ((int)sidx < cap) {
              bd[sidx] = d2;
              bi[sidx] = perm[p];
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- rank pass -> output row
    const int c = min((int)hist[bsel], cap);
    const int64_t row = (int64_t)perm[q];
    for (int ai = tid; ai < c; ai += NT) {
      const double da = bd[ai];
      const int32_t ia = bi[ai];
      const int b = bin_of<DIM>(da, thr, top0);
      const int start = b > 0 ? (int)hist[b - 1] : 0;
      if (start < K) {
        const int end = min((int)hist[b], cap);
        int rank = start;
        for (int s2 = start; s2 < end; ++s2) {
          const double db = bd[s2];
          const int32_t ib = bi[s2];
          rank += (db < da || (db == da && ib < ia)) ? 1 : 0;
        }
        if (rank < K) {
          a.out_ids[row * K + rank] = ia;
          a.out_d[row * K + rank] = sqrt(da);
        }
      }
    }
    __syncthreads();
  }
}

// Z-order levels exist for 2..kZMaxDims dimensions only (no kernels above).
template <int DIM>
constexpr bool kHasZ = DIM <= kZMaxDims;

template <int DIM, int T, bool ZL>
int occupancy_of(int threads, size_t lds) {
  int n = 0;
  KNN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_search<DIM, T, true, ZL>, threads,
                                                       lds));
  return n;
}

template <int DIM, bool ZL>
int occupancy_dim_z(int T, int threads, size_t lds) {
  switch (T) {
    case 1: return occupancy_of<DIM, 1, ZL>(threads, lds);
    case 2: return occupancy_of<DIM, 2, ZL>(threads, lds);
    case 4: return occupancy_of<DIM, 4, ZL>(threads, lds);
    case 8: return occupancy_of<DIM, 8, ZL>(threads, lds);
    case 16: return occupancy_of<DIM, 16, ZL>(threads, lds);
    case 32: return occupancy_of<DIM, 32, ZL>(threads, lds);
    default: return occupancy_of<DIM, 64, ZL>(threads, lds);
  }
}

template <int DIM>
int occupancy_dim(int T, int threads, size_t lds, bool zl) {
  if constexpr (kHasZ<DIM>) {
    if (zl) return occupancy_dim_z<DIM, true>(T, threads, lds);
  }
  KNN_CHECK(!zl, KNN_EINTERNAL, "no Z-order search kernel for this dimension");
  return occupancy_dim_z<DIM, false>(T, threads, lds);
}

template <int DIM, bool OFF32, bool ZL>
void launch_dim_off(const SearchArgs& a, int T, int blocks, int threads, size_t lds,
                    hipStream_t s) {
  switch (T) {
    case 1: k_search<DIM, 1, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 2: k_search<DIM, 2, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 4: k_search<DIM, 4, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 8: k_search<DIM, 8, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 16: k_search<DIM, 16, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 32: k_search<DIM, 32, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    case 64: k_search<DIM, 64, OFF32, ZL><<<blocks, threads, lds, s>>>(a); break;
    default: throw Error(KNN_EINVAL, "lanes_per_query must be a power of two in [1, 64]");
  }
}

template <int DIM, bool ZL>
void launch_dim_z(const SearchArgs& a, int T, int blocks, int threads, size_t lds,
                  hipStream_t s) {
  if (a.N * point_stride(DIM) * (int64_t)sizeof(double) < ((int64_t)1 << 32))
    launch_dim_off<DIM, true, ZL>(a, T, blocks, threads, lds, s);
  else
    launch_dim_off<DIM, false, ZL>(a, T, blocks, threads, lds, s);
}

template <int DIM>
void launch_dim(const SearchArgs& a, int T, int blocks, int threads, size_t lds, hipStream_t s) {
  if constexpr (kHasZ<DIM>) {
    if (a.zl) return launch_dim_z<DIM, true>(a, T, blocks, threads, lds, s);
  }
  KNN_CHECK(!a.zl, KNN_EINTERNAL, "no Z-order search kernel for this dimension");
  launch_dim_z<DIM, false>(a, T, blocks, threads, lds, s);
}

template <int DIM>
void launch_heavy_dim(const SearchArgs& a, int blocks, size_t lds, hipStream_t s) {
  if constexpr (kHasZ<DIM>) {
    if (a.zl) {
      k_search_heavy<DIM, true><<<blocks, kHeavyThreads, lds, s>>>(a);
      return;
    }
  }
  KNN_CHECK(!a.zl, KNN_EINTERNAL, "no Z-order search kernel for this dimension");
  k_search_heavy<DIM, false><<<blocks, kHeavyThreads, lds, s>>>(a);
}

}  // namespace

void launch_defer_filter(const DeferArgs& a, int dims, hipStream_t s) {
  if (a.n_active <= 0) {
    launch_zero(a.out_count, sizeof(uint32_t), s);
    return;
  }
  const int64_t nb = ceil_div(a.n_active, kDeferTile);
  // the tile area: nb counts (padded to even), then 2 masks per 64 slots
  const int64_t cwords = (nb + 2) & ~(int64_t)1;
  const int64_t mwords = nb * 4 * kDeferRounds * 4;
  DeferArgs b = a;
  b.tile_counts = scan_tile_area(a.state, a.state_elems, cwords + mwords);
  b.tile_masks = b.tile_counts + cwords;
  switch (dims) {
    case 2: k_defer_filter<2><<<(unsigned)nb, 256, 0, s>>>(b); break;
    case 3: k_defer_filter<3><<<(unsigned)nb, 256, 0, s>>>(b); break;
    case 4: k_defer_filter<4><<<(unsigned)nb, 256, 0, s>>>(b); break;
    case 5: k_defer_filter<5><<<(unsigned)nb, 256, 0, s>>>(b); break;
    case 6: k_defer_filter<6><<<(unsigned)nb, 256, 0, s>>>(b); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
  launch_exclusive_scan(b.tile_counts, b.tile_counts, nb, a.out_count, a.state, a.state_elems, s);
  k_defer_write<<<(unsigned)nb, 256, 0, s>>>(b);
  KNN_LAUNCHED();
}

static size_t lds_base_per_wave(int dims, int T, int cap, bool zl) {
  const int G = 64 / T;
  size_t R = 1;
  for (int j = 0; j < (zl ? dims : dims - 1); ++j) R *= 3;
  return (size_t)cap * G * (sizeof(double) + sizeof(int32_t)) +
         (size_t)(NB + 1) * G * sizeof(uint32_t) + (size_t)kFailBuf * sizeof(int32_t) +
         2 * (R + 1) * G * sizeof(uint32_t);
}

// Speculative slots per query: twice the survivor buffer, but only what the
// per-wave budget of 16 KiB leaves beside the other buffers; none when that
// is below cap (a speculation needs room for more than K).
int search_spec_slots(int dims, int T, int cap, bool zl) {
  const int G = 64 / T;
  const size_t base = lds_base_per_wave(dims, T, cap, zl);
  const int room = base < 16384 ? (int)((16384 - base) / (G * sizeof(uint32_t))) : 0;
  const int sc = std::min(2 * cap, room);
  return sc >= cap ? sc : 0;
}

// Coefficient of the predicted K-th squared distance, coef * C^(-2/n) for C
// points in the 3^n block of cells of side w: w^2 (K 3^n / V_n)^(2/n) with V_n
// the volume of the unit n-ball.  The speculation limit takes it times
// 1.7^(2/n) (the kept set then holds about 1.7 K points at uniform density);
// a query is deferred when the prediction exceeds thr by 1.3, i.e. its
// product with 1/1.3 exceeds thr (measured offline on
// exponential 2-D and 4-D data at level 0: half of all queries, 84 % of the
// failures, 0.1 % of the successes).
double search_density_coef(int dims, int K, double w) {
  const double n = dims;
  const double vn = std::pow(M_PI, n / 2) / std::tgamma(n / 2 + 1);
  return w * w * std::pow(K * std::pow(3.0, n) / vn, 2.0 / n);
}

size_t search_lds_per_wave(int dims, int T, int cap, bool zl) {
  return lds_base_per_wave(dims, T, cap, zl) +
         (size_t)(64 / T) * search_spec_slots(dims, T, cap, zl) * sizeof(uint32_t);
}

int search_waves_per_block(int dims, int T, int cap, bool zl) {
  size_t per = search_lds_per_wave(dims, T, cap, zl);
  int w = (int)(65536 / per);
  if (w > 4) w = 4;
  if (w < 1) w = 1;
  return w;
}

int search_blocks_per_cu(int dims, int T, int cap, bool zl) {
  // the occupancy query costs host time on every call; levels ask it often
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, int, bool>, int> cache;
  int dev = 0;
  KNN_HIP(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, dims, T, cap, zl);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const int waves = search_waves_per_block(dims, T, cap, zl);
  const size_t lds = search_lds_per_wave(dims, T, cap, zl) * waves;
  int n = 1;
  switch (dims) {
    case 2: n = occupancy_dim<2>(T, waves * 64, lds, zl); break;
    case 3: n = occupancy_dim<3>(T, waves * 64, lds, zl); break;
    case 4: n = occupancy_dim<4>(T, waves * 64, lds, zl); break;
    case 5: n = occupancy_dim<5>(T, waves * 64, lds, zl); break;
    case 6: n = occupancy_dim<6>(T, waves * 64, lds, zl); break;
    default: break;
  }
  n = n > 0 ? n : 1;
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = n;
  return n;
}

void launch_search_heavy(const SearchArgs& a, int dims, int blocks, hipStream_t s) {
  KNN_CHECK(a.heavy && a.n_heavy && blocks > 0, KNN_EINTERNAL, "heavy-query launch without a list");
  const size_t lds = (size_t)a.cap * (sizeof(double) + sizeof(int32_t));
  KNN_CHECK(lds <= 49152, KNN_EINVAL, "K too large for the per-query buffers");
  switch (dims) {
    case 2: launch_heavy_dim<2>(a, blocks, lds, s); break;
    case 3: launch_heavy_dim<3>(a, blocks, lds, s); break;
    case 4: launch_heavy_dim<4>(a, blocks, lds, s); break;
    case 5: launch_heavy_dim<5>(a, blocks, lds, s); break;
    case 6: launch_heavy_dim<6>(a, blocks, lds, s); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
}

void launch_search(const SearchArgs& a, int dims, int T, int grid_blocks, hipStream_t s) {
  KNN_CHECK(a.cap >= NB2 / 2 + 1, KNN_EINTERNAL, "per-query buffer too small");
  const int waves = search_waves_per_block(dims, T, a.cap, a.zl != 0);
  const size_t lds = search_lds_per_wave(dims, T, a.cap, a.zl != 0) * waves;
  KNN_CHECK(lds <= 65536, KNN_EINVAL,
            "per-query buffers exceed the LDS (raise lanes_per_query or lower K)");
  const int threads = waves * 64;
  switch (dims) {
    case 2: launch_dim<2>(a, T, grid_blocks, threads, lds, s); break;
    case 3: launch_dim<3>(a, T, grid_blocks, threads, lds, s); break;
    case 4: launch_dim<4>(a, T, grid_blocks, threads, lds, s); break;
    case 5: launch_dim<5>(a, T, grid_blocks, threads, lds, s); break;
    case 6: launch_dim<6>(a, T, grid_blocks, threads, lds, s); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
}

}  // namespace knn
