// epsjoin.hip -- kernels of the distance similarity self-join the method
// builds on (every pair within a search distance eps; Sec. 1 and Sec. 3): a
// count pass and a write pass over one grid level whose 3^n block around a
// query's cell holds its whole eps-ball (Sec. 3.1), an exclusive 64-bit
// prefix of the counts, and the query ranges of result batches that fit a
// buffer (the batching scheme of Sec. 3.2, with exact counts).
#pragma clang fp contract(off)

#include "kernels.hpp"

namespace knn {

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                     // counts per thread in the prefix
constexpr int64_t kScanTile = kBlock * kScanItems;  // counts per prefix tile
// A part of a segment is skipped when its lower bound b satisfies
// b * (1 - 2^-40) > t: the factor covers the rounding of the bound and of
// every candidate's computed d^2 (a few ulps each).
constexpr double kSkipShrink = 1.0 - 0x1p-40;

template <int DIM>
__device__ __forceinline__ double pt_d2(const double* __restrict__ Xs, uint32_t p,
                                        const double (&q)[DIM]) {
  constexpr int S = point_stride(DIM);
  const double2* src = reinterpret_cast<const double2*>(Xs + (size_t)p * S);
  double s = 0.0;
#pragma unroll
  for (int h = 0; h < S / 2; ++h) {
    const double2 t2 = src[h];
    const double a = __dsub_rn(t2.x, q[2 * h]);
    s = __dadd_rn(s, __dmul_rn(a, a));
    if (2 * h + 1 < DIM) {
      const double b = __dsub_rn(t2.y, q[2 * h + 1]);
      s = __dadd_rn(s, __dmul_rn(b, b));
    }
  }
  return s;
}

// One group of T lanes per query (sorted position p = slot * stride).
// WRITE = false: cnt[slot] = the points v != p of the 3^n block with
// d^2 <= t.  WRITE = true (stride 1): the pairs of the positions [first,
// last) at out + off[p] - off[first], in the order of the cell's row segments
// and of the sorted positions inside each; every trip count of a group is
// the same for its lanes, so a hit's slot is the group's running count plus
// its rank in the group's ballot.  Both passes skip exactly the same parts of
// the segments (the same code on the same values), so the write pass finds
// the counted pairs; a write beyond the query's counted slots is dropped all
// the same.
template <int DIM, int T, bool WRITE>
__global__ void __launch_bounds__(kBlock)
k_eps_pass(const double* __restrict__ Xs, int64_t N, const int32_t* __restrict__ perm,
           const uint32_t* __restrict__ cell_of, const uint32_t* __restrict__ ranges,
           const uint8_t* __restrict__ rslot, const uint32_t* __restrict__ nrng, int R,
           GridGeom gg, double w, double margin, double t, int64_t stride, int64_t first,
           int64_t last, uint32_t* __restrict__ cnt_out, const uint64_t* __restrict__ off,
           int32_t* __restrict__ out_q, int32_t* __restrict__ out_j, double* __restrict__ out_d) {
  constexpr int G = 64 / T;
  const int lane = threadIdx.x & 63;
  const int g = lane / T, l = lane % T;
  const uint64_t gmask = T == 64 ? ~0ull : (((1ull << T) - 1ull) << (g * T));
  const uint64_t lane_lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t nq = WRITE ? last - first : (N + stride - 1) / stride;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t wv = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; wv * G < nq;
       wv += waves) {
    const int64_t slot = wv * G + g;
    const bool in = slot < nq;
    const int64_t q = in ? (WRITE ? first + slot : slot * stride) : 0;
    double qx[DIM];
    {
      constexpr int S = point_stride(DIM);
      const double2* src = reinterpret_cast<const double2*>(Xs + (size_t)q * S);
#pragma unroll
      for (int h = 0; h < S / 2; ++h) {
        const double2 t2 = src[h];
        qx[2 * h] = t2.x;
        if (2 * h + 1 < DIM) qx[2 * h + 1] = t2.y;
      }
    }
    // lower bounds of the distance from the query to the faces of its cell
    // (the cell coordinates carry at most `margin` cells of rounding each)
    double flo[DIM], fhi[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      const double u = __dmul_rn(__dsub_rn(qx[j], gg.lo[j]), gg.inv_w);
      const double fr = u - floor(u);  // exact
      flo[j] = fmax(fr - margin, 0.0) * w;
      fhi[j] = fmax((1.0 - fr) - margin, 0.0) * w;
    }
    const double dlo = flo[DIM - 1] * flo[DIM - 1], dhi = fhi[DIM - 1] * fhi[DIM - 1];
    const uint32_t cell = cell_of[q];
    const int nr = in ? (int)nrng[cell] : 0;
    const uint32_t* rg = ranges + (size_t)cell * R * 4;
    const uint8_t* rs = rslot + (size_t)cell * R;
    int32_t id = 0;
    uint64_t base = 0, lim = 0;
    if (WRITE && in) {
      id = perm[q];
      const uint64_t o0 = off[first];
      base = off[q] - o0;
      lim = off[q + 1] - o0;
    }
    uint32_t cnt = 0;  // the group's running count (WRITE) or the lane's
    for (int r = 0; r < nr; ++r) {
      const uint4 r4 = reinterpret_cast<const uint4*>(rg)[r];  // start, mid0, mid1, end
      double b0 = 0.0;
      {
        int rr = rs[r];
#pragma unroll
        for (int j = DIM - 2; j >= 0; --j) {
          const int o = rr % 3;
          rr /= 3;
          const double d = o == 0 ? flo[j] : (o == 2 ? fhi[j] : 0.0);
          b0 += d * d;
        }
      }
      if (b0 * kSkipShrink > t) continue;
      const uint32_t st = (b0 + dlo) * kSkipShrink <= t ? r4.x : r4.y;
      const uint32_t en = (b0 + dhi) * kSkipShrink <= t ? r4.w : r4.z;
      for (uint32_t vb = st; vb < en; vb += T) {
        const uint32_t v = vb + (uint32_t)l;
        bool hit = false;
        double d2 = 0.0;
        if (v < en && v != (uint32_t)q) {
          d2 = pt_d2<DIM>(Xs, v, qx);
          hit = d2 <= t;
        }
        if (WRITE) {
          const uint64_t hm = __ballot(hit) & gmask;
          if (hit) {
            const uint64_t k = base + cnt + (uint64_t)__popcll(hm & lane_lt);
            if (k < lim) {
              out_q[k] = id;
              out_j[k] = perm[v];
              out_d[k] = sqrt(d2);
            }
          }
          cnt += (uint32_t)__popcll(hm);
        } else {
          cnt += hit ? 1u : 0u;
        }
      }
    }
    if (!WRITE) {
#pragma unroll
      for (int o = 1; o < T; o <<= 1) cnt += __shfl_xor(cnt, o, 64);
      if (in && l == 0) cnt_out[slot] = cnt;
    }
  }
}

// Exclusive prefix of n uint32 counts into n + 1 uint64 offsets, in three
// launches: tile sums, a one-block scan of the tile sums, and the tiles.
__global__ void __launch_bounds__(kBlock)
k_tile_sums(const uint32_t* __restrict__ c, int64_t n, uint64_t* __restrict__ tile) {
  __shared__ uint64_t red[kBlock / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
  for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
    const int64_t p = t0 + i;
    if (p < n) s += c[p];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (int i = 0; i < kBlock / 64; ++i) tot += red[i];
    tile[blockIdx.x] = tot;
  }
}

__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t* total) {
  __shared__ uint64_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wi = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) wsum[wi] = inc;
  __syncthreads();
  uint64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < wi) before += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// One block: tile[i] <- the sum of tiles before i; tile[nt] <- the total.
__global__ void __launch_bounds__(kBlock) k_tile_scan(uint64_t* __restrict__ tile, int64_t nt) {
  uint64_t carry = 0;
  for (int64_t b = 0; b < nt; b += kBlock) {
    const int64_t i = b + threadIdx.x;
    const uint64_t v = i < nt ? tile[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan64(v, &tot);
    if (i < nt) tile[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) tile[nt] = carry;
}

__global__ void __launch_bounds__(kBlock)
k_tile_apply(const uint32_t* __restrict__ c, int64_t n, const uint64_t* __restrict__ tile,
             int64_t nt, uint64_t* __restrict__ off) {
  const int64_t p0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = p0 + i < n ? c[p0 + i] : 0u;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = tile[blockIdx.x] + block_excl_scan64(s, &tot);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (p0 + i < n) off[p0 + i] = run;
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = tile[nt];
}

// Greedy batches from position `first`: batch b ends at the largest e with
// off[e] - off[start] <= cap (start = the previous batch's end); at most maxb
// batches, stopping at n.  bounds[2b] = e, bounds[2b+1] = off[e].
// status[0] = the number of batches written, or -1 when the position at which
// a batch would start alone holds more than cap pairs (status[2] = its pair
// count); status[1] = off[first].
__global__ void k_batch_bounds(const uint64_t* __restrict__ off, int64_t n, int64_t first,
                               uint64_t cap, int64_t maxb, int64_t* __restrict__ bounds,
                               int64_t* __restrict__ status) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  status[1] = (int64_t)off[first];
  status[2] = 0;
  int64_t s = first, nb = 0;
  while (s < n && nb < maxb) {
    const uint64_t lim = off[s] + cap;
    // off is non-decreasing: the largest e in [s, n] with off[e] <= lim
    int64_t lo = s, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (off[mid] <= lim) lo = mid;
      else hi = mid - 1;
    }
    if (lo == s) {
      status[0] = -1;
      status[2] = (int64_t)(off[s + 1] - off[s]);
      return;
    }
    bounds[2 * nb] = lo;
    bounds[2 * nb + 1] = (int64_t)off[lo];
    ++nb;
    s = lo;
  }
  status[0] = nb;
}

__global__ void k_counts_by_id(const uint32_t* __restrict__ c, const int32_t* __restrict__ perm,
                               int64_t n, int32_t* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    out[perm[p]] = (int32_t)c[p];
}

template <int DIM, int T, bool WRITE>
void eps_launch(const EpsPassArgs& a, hipStream_t s) {
  const int64_t nq = WRITE ? a.last - a.first : ceil_div(a.N, a.stride);
  if (nq <= 0) return;
  constexpr int G = 64 / T;
  const int64_t waves = ceil_div(nq, G);
  const int blocks = (int)std::min<int64_t>(ceil_div(waves, kBlock / 64), 1 << 20);
  k_eps_pass<DIM, T, WRITE><<<blocks, kBlock, 0, s>>>(
      a.Xs, a.N, a.perm, a.cell_of, a.ranges, a.rslot, a.nrng, a.R, a.gg, a.w, a.margin, a.t,
      a.stride, a.first, a.last, a.counts, a.off, a.out_q, a.out_j, a.out_d);
  KNN_LAUNCHED();
}

template <bool WRITE>
void eps_dispatch(const EpsPassArgs& a, hipStream_t s) {
  switch (a.gg.dims) {
    case 2: eps_launch<2, 8, WRITE>(a, s); break;
    case 3: eps_launch<3, 8, WRITE>(a, s); break;
    case 4: eps_launch<4, 16, WRITE>(a, s); break;
    case 5: eps_launch<5, 16, WRITE>(a, s); break;
    case 6: eps_launch<6, 16, WRITE>(a, s); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
}

}  // namespace

void launch_eps_count(const EpsPassArgs& a, hipStream_t s) {
  KNN_CHECK(a.stride >= 1, KNN_EINTERNAL, "count stride must be >= 1");
  eps_dispatch<false>(a, s);
}

void launch_eps_write(const EpsPassArgs& a, hipStream_t s) {
  KNN_CHECK(a.first >= 0 && a.first <= a.last && a.last <= a.N, KNN_EINTERNAL,
            "write pass: position range outside [0, N]");
  eps_dispatch<true>(a, s);
}

int64_t eps_scan_tiles(int64_t n) { return ceil_div(std::max<int64_t>(n, 1), kScanTile) + 1; }

void launch_offsets(const uint32_t* counts, int64_t n, uint64_t* tiles, uint64_t* off,
                    hipStream_t s) {
  const int64_t nt = ceil_div(std::max<int64_t>(n, 1), kScanTile);
  k_tile_sums<<<(int)nt, kBlock, 0, s>>>(counts, n, tiles);
  KNN_LAUNCHED();
  k_tile_scan<<<1, kBlock, 0, s>>>(tiles, nt);
  KNN_LAUNCHED();
  k_tile_apply<<<(int)nt, kBlock, 0, s>>>(counts, n, tiles, nt, off);
  KNN_LAUNCHED();
}

void launch_batch_bounds(const uint64_t* off, int64_t n, int64_t first, uint64_t cap,
                         int64_t maxb, int64_t* bounds, int64_t* status, hipStream_t s) {
  k_batch_bounds<<<1, 64, 0, s>>>(off, n, first, cap, maxb, bounds, status);
  KNN_LAUNCHED();
}

void launch_counts_by_id(const uint32_t* counts, const int32_t* perm, int64_t n, int32_t* out,
                         hipStream_t s) {
  if (n <= 0) return;
  k_counts_by_id<<<(int)std::min<int64_t>(ceil_div(n, kBlock), 8192), kBlock, 0, s>>>(counts, perm,
                                                                                     n, out);
  KNN_LAUNCHED();
}

}  // namespace knn
