// grid.hip -- construction of one uniform-grid level on the GPU (Sec. 3.1,
// built on the GPU as in Sec. 4.6): layout change, bounds, cell keys, LSD
// radix sort, cell table by flag + exclusive scan, SoA gather of the sorted
// coordinates, and the row-segment neighbour ranges of every non-empty cell.
// Also the small helpers of the level loop (work-item keys, failure flags).
#pragma clang fp contract(off)

#include "kernels.hpp"
#include "lookback.hpp"

namespace knn {

namespace {

constexpr int kBlock = 256;

__device__ inline int64_t cell_coord(double x, double lo, double inv_w) {
  // floor((x - lo) * inv_w), both operations rounded (no contraction)
  return (int64_t)floor(__dmul_rn(__dsub_rn(x, lo), inv_w));
}

// --------------------------------------------------------------------------
// layout + bounds
// --------------------------------------------------------------------------
__global__ void k_aos_to_soa(const double* __restrict__ D, int64_t N, int n,
                             double* __restrict__ X, uint32_t* bad) {
  uint32_t nbad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = D[e];
    int64_t i = e / n;
    int j = (int)(e - i * n);
    X[(int64_t)j * N + i] = v;
    if (!isfinite(v)) ++nbad;
  }
  if (nbad) atomicAdd(bad, nbad);
}

__global__ void k_bounds_partial(const double* __restrict__ X, int64_t N, int n,
                                 double* __restrict__ part) {
  __shared__ double smin[kBlock], smax[kBlock];
  for (int j = 0; j < n; ++j) {
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
      double v = X[(int64_t)j * N + i];
      mn = fmin(mn, v);
      mx = fmax(mx, v);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[(2 * j) * gridDim.x + blockIdx.x] = smin[0];
      part[(2 * j + 1) * gridDim.x + blockIdx.x] = smax[0];
    }
    __syncthreads();
  }
}

__global__ void k_bounds_final(const double* __restrict__ part, int nparts, int n,
                               double* lo, double* hi) {
  __shared__ double smin[kBlock], smax[kBlock];
  for (int j = 0; j < n; ++j) {
    double mn = INFINITY, mx = -INFINITY;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
      mn = fmin(mn, part[(2 * j) * nparts + i]);
      mx = fmax(mx, part[(2 * j + 1) * nparts + i]);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      lo[j] = smin[0];
      hi[j] = smax[0];
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// exclusive scan of uint32
// --------------------------------------------------------------------------

constexpr int kOneItems = 32;
constexpr int kOneTile = kBlock * kOneItems;
static_assert(kOneTile >= kLbMinTile, "scan state sized for larger tiles");

// Single-pass exclusive scan (look-back over tile words, lookback.hpp).
template <bool VEC>
__global__ void __launch_bounds__(kBlock)
k_scan_onepass(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n, int64_t nb,
               uint32_t* __restrict__ state, uint32_t* __restrict__ total) {
  __shared__ uint32_t s_excl;
  const LbTile lt = lb_take_tile(state, nb);
  // thread t owns kOneItems consecutive elements of the tile
  const int64_t base = lt.tile * kOneTile + (int64_t)threadIdx.x * kOneItems;
  const bool whole = VEC && base + kOneItems <= n;
  uint32_t v[kOneItems];
  if (whole) {
#pragma unroll
    for (int k = 0; k < kOneItems / 4; ++k) {
      const uint4 q = reinterpret_cast<const uint4*>(in + base)[k];
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) v[k] = base + k < n ? in[base + k] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kOneItems; ++k) sum += v[k];
  uint32_t agg;
  uint32_t ex = block_excl_scan<kBlock>(sum, &agg);
  const uint32_t excl = lb_tile_prefix(state, lt, agg, &s_excl);
  if (threadIdx.x == 0 && lt.tile == nb - 1 && total) *total = excl + agg;
  ex += excl;
  if (whole) {
#pragma unroll
    for (int k = 0; k < kOneItems / 4; ++k) {
      uint4 q;
      q.x = ex;
      ex += v[4 * k];
      q.y = ex;
      ex += v[4 * k + 1];
      q.z = ex;
      ex += v[4 * k + 2];
      q.w = ex;
      ex += v[4 * k + 3];
      reinterpret_cast<uint4*>(out + base)[k] = q;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kOneItems; ++k) {
      if (base + k < n) out[base + k] = ex;
      ex += v[k];
    }
  }
}

// --------------------------------------------------------------------------
// LSD radix sort, DB-bit digits (8 or 11): per-tile histogram, scan, stable
// scatter.  Within a tile, a key's rank among equal digits comes from DB wave
// ballots (lanes with the same digit) plus the counts of earlier waves and
// earlier chunks of the tile, so equal digits keep their input order.
// --------------------------------------------------------------------------
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kMaxDigitBits = 11;

template <int DB, class KeyT>
__global__ void k_radix_hist(const KeyT* __restrict__ keys, int64_t n, int shift,
                             uint32_t* __restrict__ hist, int64_t nb) {
  constexpr int RB = 1 << DB;
  __shared__ uint32_t h[RB];
  for (int d = threadIdx.x; d < RB; d += kBlock) h[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int k = 0; k < kRadixItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (uint32_t)(RB - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RB; d += kBlock) hist[(int64_t)d * nb + blockIdx.x] = h[d];
}

// Stable scatter of one tile: rounds of kBlock keys in input order; in a
// round, a key's rank among the wave's keys of its digit comes from DB
// ballots, and the wave's count per digit goes to wcnt[w][d] (written by the
// digit's first lane), so the keys of earlier waves precede it.  Only the
// entries a round touched are updated afterwards (run[d] advanced, wcnt
// cleared), not all RB digits.
template <int DB, class KeyT>
__global__ void k_radix_scatter(const KeyT* __restrict__ keys,
                                const int32_t* __restrict__ vals, int64_t n, int shift,
                                const uint32_t* __restrict__ offs, int64_t nb,
                                KeyT* __restrict__ okeys, int32_t* __restrict__ ovals) {
  constexpr int RB = 1 << DB;
  __shared__ uint32_t run[RB];
  __shared__ uint32_t wcnt[kBlock / 64][RB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int d = t; d < RB; d += kBlock) {
    run[d] = offs[(int64_t)d * nb + blockIdx.x];
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) wcnt[i][d] = 0;
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int k = 0; k < kRadixItems; ++k) {
    int64_t i = base + (int64_t)k * kBlock + t;
    bool valid = i < n;
    KeyT key = valid ? keys[i] : 0;
    int32_t val = valid ? vals[i] : 0;
    uint32_t d = (uint32_t)(key >> shift) & (uint32_t)(RB - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const bool leader = valid && rank == 0;
    const uint32_t cnt = (uint32_t)__popcll(peers);
    if (leader) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int i2 = 0; i2 < w; ++i2) pos += wcnt[i2][d];
      okeys[pos] = key;
      ovals[pos] = val;
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&run[d], cnt);
      wcnt[w][d] = 0;
    }
    __syncthreads();
  }
}

// Stable scatter through LDS (8-bit digits): the tile's keys are first placed
// in LDS in digit order (the same ballot ranks as above, with tile-local
// digit starts), then written out digit run by digit run, so consecutive
// lanes write consecutive addresses of one run (about 16 keys per run for a
// 4096-key tile) instead of 256 scattered 8-byte stores per round.  The tile's
// count of digit d is the difference of consecutive entries of the scanned
// (digit-major, tile-minor) offsets, the last one closing at n.
template <class KeyT>
__global__ void __launch_bounds__(kBlock)
k_radix_scatter_lds(const KeyT* __restrict__ keys, const int32_t* __restrict__ vals,
                    int64_t n, int shift, const uint32_t* __restrict__ offs, int64_t nb,
                    KeyT* __restrict__ okeys, int32_t* __restrict__ ovals) {
  constexpr int DB = 8;
  constexpr int RB = 1 << DB;
  static_assert(RB == kBlock, "one digit per thread in the tile scan");
  __shared__ KeyT sk[kRadixTile];
  __shared__ int32_t sv[kRadixTile];
  __shared__ uint32_t lfirst[RB], lrun[RB], gbase[RB];
  __shared__ uint32_t wcnt[kBlock / 64][RB];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  {
    const int64_t e = (int64_t)t * nb + blockIdx.x;
    const uint32_t o = offs[e];
    const uint32_t nx = e + 1 < (int64_t)RB * nb ? offs[e + 1] : (uint32_t)n;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<kBlock>(nx - o, &tot);
    lfirst[t] = ex;
    lrun[t] = ex;
    gbase[t] = o;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) wcnt[i][t] = 0;
  }
  // the tile's keys and values, all loads in flight at once (the rounds
  // below would otherwise wait for one load each)
  KeyT kk[kRadixItems];
  int32_t vv[kRadixItems];
#pragma unroll
  for (int k = 0; k < kRadixItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + t;
    kk[k] = i < n ? keys[i] : 0;
    vv[k] = i < n ? vals[i] : 0;
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int k = 0; k < kRadixItems; ++k) {
    const int64_t i = base + (int64_t)k * kBlock + t;
    const bool valid = i < n;
    const KeyT key = kk[k];
    const int32_t val = vv[k];
    const uint32_t d = (uint32_t)(key >> shift) & (uint32_t)(RB - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const bool leader = valid && rank == 0;
    const uint32_t cnt = (uint32_t)__popcll(peers);
    if (leader) wcnt[w][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t pos = lrun[d] + rank;
      for (int i2 = 0; i2 < w; ++i2) pos += wcnt[i2][d];
      sk[pos] = key;
      sv[pos] = val;
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&lrun[d], cnt);  // one leader per digit and wavefront
      wcnt[w][d] = 0;
    }
    __syncthreads();
  }
  const int64_t tn = n - base < (int64_t)kRadixTile ? n - base : (int64_t)kRadixTile;
  for (int j = t; j < (int)tn; j += kBlock) {
    const KeyT key = sk[j];
    const uint32_t d = (uint32_t)(key >> shift) & (uint32_t)(RB - 1);
    const uint32_t pos = gbase[d] + ((uint32_t)j - lfirst[d]);
    okeys[pos] = key;
    ovals[pos] = sv[j];
  }
}

// --------------------------------------------------------------------------
// grid level
// --------------------------------------------------------------------------
struct GeomDev {
  double lo[kMaxDims];
  double inv_w;
  uint64_t stride[kMaxDims];
  uint64_t rstride[kMaxDims];  // row index stride (stride / g_last) of the first n-1 dims
  int64_t g[kMaxDims];
  int32_t zbits;               // > 0: Z-order keys with this many bits per dimension
};

// Z-order key of cell coordinates c (bits bits each): bit b of dimension j
// goes to position b*DIM + DIM-1-j.
template <int DIM>
__device__ inline uint64_t zorder_key(const int64_t (&c)[DIM], int bits) {
  uint64_t key = 0;
  for (int b = bits - 1; b >= 0; --b) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) key = (key << 1) | (((uint64_t)c[j] >> b) & 1ull);
  }
  return key;
}

template <int DIM>
__device__ inline void zorder_coords(uint64_t key, int bits, int64_t (&c)[DIM]) {
#pragma unroll
  for (int j = 0; j < DIM; ++j) c[j] = 0;
  for (int b = bits - 1; b >= 0; --b) {
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      c[j] |= (int64_t)((key >> (b * DIM + DIM - 1 - j)) & 1ull) << b;
  }
}

GeomDev to_dev(const GridGeom& gg) {
  GeomDev d{};
  for (int j = 0; j < kMaxDims; ++j) {
    d.lo[j] = gg.lo[j];
    d.stride[j] = gg.stride[j];
    d.rstride[j] = (j < gg.dims - 1 && gg.g[gg.dims - 1] > 0)
                       ? gg.stride[j] / (uint64_t)gg.g[gg.dims - 1] : 0;
    d.g[j] = gg.g[j];
  }
  d.inv_w = gg.inv_w;
  d.zbits = gg.zbits;
  return d;
}

template <int DIM, class KeyT>
__global__ void k_cell_keys(const double* __restrict__ X, int64_t N, GeomDev gd,
                            KeyT* __restrict__ keys, int32_t* __restrict__ vals) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t key = 0;
    if (gd.zbits > 0) {
      int64_t c[DIM];
#pragma unroll
      for (int j = 0; j < DIM; ++j) c[j] = cell_coord(X[(int64_t)j * N + i], gd.lo[j], gd.inv_w);
      key = zorder_key<DIM>(c, gd.zbits);
    } else {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
        key += (uint64_t)cell_coord(X[(int64_t)j * N + i], gd.lo[j], gd.inv_w) * gd.stride[j];
    }
    keys[i] = (KeyT)key;
    vals[i] = (int32_t)i;
  }
}

// Keys of the previous level's sorted points (point-major), their positions
// as values: a level sorted from there reads and writes far more coherently
// than from the original order.
template <int DIM>
__global__ void k_cell_keys_points(const double* __restrict__ Xs, int64_t N, GeomDev gd,
                                   uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  constexpr int S = point_stride(DIM);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double2* src = reinterpret_cast<const double2*>(Xs + i * S);
    double x[S];
#pragma unroll
    for (int h = 0; h < S / 2; ++h) {
      const double2 t = src[h];
      x[2 * h] = t.x;
      x[2 * h + 1] = t.y;
    }
    uint64_t key = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      key += (uint64_t)cell_coord(x[j], gd.lo[j], gd.inv_w) * gd.stride[j];
    keys[i] = key;
    vals[i] = (int32_t)i;
  }
}

// New sorted order from previous positions: point p' takes the previous
// point pos[p'] (coordinates and id).
__global__ void k_gather_prev(const double* __restrict__ Xs_prev, const int32_t* __restrict__ perm_prev,
                              const int32_t* __restrict__ pos, int64_t N, int S,
                              double* __restrict__ Xs, int32_t* __restrict__ perm) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = pos[p];
    perm[p] = perm_prev[src];
    const double2* in = reinterpret_cast<const double2*>(Xs_prev + src * S);
    double2* out = reinterpret_cast<double2*>(Xs + p * S);
    for (int h = 0; h < S / 2; ++h) out[h] = in[h];
  }
}

// Cell table: a cell starts where the sorted key changes.  A tile is
// kCtRounds rounds of 64 consecutive positions per wavefront (coalesced); the
// start flags of a round are one ballot.  Three launches: the tiles' start
// counts, their exclusive scan, and a second sweep that emits every start's
// cell key and first position and every position's cell (offsets: the tile's
// scanned count plus the block's earlier wavefronts and the ballot prefix).
// No block waits for another, and the tile counts are plain loads and stores.
// The last position writes M and cell_start[M].
constexpr int kCtRounds = 16;
constexpr int kCtTile = kBlock * kCtRounds;

// Exclusive prefix of this wavefront's count over the block's wavefronts
// (all threads; one barrier); *agg = the block's total.
__device__ inline uint32_t block_wave_prefix(uint32_t wcount, uint32_t* agg) {
  __shared__ uint32_t s_w[kBlock / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_w[w] = wcount;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < w) before += s_w[i];
    tot += s_w[i];
  }
  *agg = tot;
  return before;
}

// WRITE = false: tile_words[tile] = the tile's cell starts; WRITE = true:
// tile_words[tile] holds the starts of all earlier tiles.
template <bool WRITE, class KeyT>
__global__ void __launch_bounds__(kBlock)
k_cell_table(const KeyT* __restrict__ keys, int64_t N, int shift,
             uint32_t* __restrict__ cell_of, uint64_t* __restrict__ cell_key,
             uint32_t* __restrict__ cell_start, uint32_t* __restrict__ d_M,
             uint32_t* __restrict__ tile_words) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbase = (int64_t)blockIdx.x * kCtTile + (int64_t)w * 64 * kCtRounds;
  uint64_t key[kCtRounds], m[kCtRounds];
  uint32_t cnt = 0;
#pragma unroll
  for (int r = 0; r < kCtRounds; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    // widened before the shift (the shift may equal a 32-bit key's width)
    key[r] = i < N ? (uint64_t)keys[i] >> shift : 0;
    const uint64_t up = __shfl_up(key[r], 1, 64);
    const uint64_t prev = lane > 0 ? up : (i > 0 && i < N ? (uint64_t)keys[i - 1] >> shift : 0);
    m[r] = __ballot(i < N && (i == 0 || key[r] != prev));
    cnt += (uint32_t)__popcll(m[r]);
  }
  uint32_t agg;
  const uint32_t before = block_wave_prefix(cnt, &agg);
  if (!WRITE) {
    if (threadIdx.x == 0) tile_words[blockIdx.x] = agg;
    return;
  }
  uint32_t c = tile_words[blockIdx.x] + before;  // cells started before this wavefront
#pragma unroll
  for (int r = 0; r < kCtRounds; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    const bool f = (m[r] >> lane) & 1ull;
    const uint32_t ci = c + (uint32_t)__popcll(m[r] & lt_mask);  // this start's cell
    if (i < N) {
      if (f) {
        cell_key[ci] = key[r];
        cell_start[ci] = (uint32_t)i;
      }
      cell_of[i] = f ? ci : ci - 1u;
      if (i == N - 1) {
        const uint32_t M = ci + (f ? 1u : 0u);
        cell_start[M] = (uint32_t)N;
        *d_M = M;
      }
    }
    c += (uint32_t)__popcll(m[r]);
  }
}

// Active list: the sorted positions whose point failed, in order; the same
// three launches as the cell table (tile counts, scan, writes).
template <bool WRITE>
__global__ void __launch_bounds__(kBlock)
k_active_list(const uint8_t* __restrict__ failed, uint8_t tag, bool at_least,
              const int32_t* __restrict__ perm, int64_t N, int32_t base,
              int32_t* __restrict__ out, uint32_t* __restrict__ tile_words) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbase = (int64_t)blockIdx.x * kCtTile + (int64_t)w * 64 * kCtRounds;
  uint64_t m[kCtRounds];
  uint32_t cnt = 0;
#pragma unroll
  for (int r = 0; r < kCtRounds; ++r) {
    const int64_t p = wbase + r * 64 + lane;
    const uint8_t f = p < N ? failed[perm ? perm[p] : (int32_t)p] : (uint8_t)0;
    m[r] = __ballot(p < N && (at_least ? (f >= tag) : (f == tag)));
    cnt += (uint32_t)__popcll(m[r]);
  }
  uint32_t agg;
  const uint32_t before = block_wave_prefix(cnt, &agg);
  if (!WRITE) {
    if (threadIdx.x == 0) tile_words[blockIdx.x] = agg;
    return;
  }
  uint32_t o = tile_words[blockIdx.x] + before;
#pragma unroll
  for (int r = 0; r < kCtRounds; ++r) {
    if ((m[r] >> lane) & 1ull)
      out[o + (uint32_t)__popcll(m[r] & lt_mask)] = base + (int32_t)(wbase + r * 64 + lane);
    o += (uint32_t)__popcll(m[r]);
  }
}

// Point-major sorted coordinates: point p (sorted position) takes the row
// perm[p] of the row-major copy, padded to an even count with 0.
__global__ void k_gather_points(const double* __restrict__ XA, const int32_t* __restrict__ perm,
                                int64_t N, int n, double* __restrict__ Xs) {
  const int S = point_stride(n);
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = perm[p];
    const double* in = XA + src * n;
    double2* out = reinterpret_cast<double2*>(Xs + p * S);
    for (int h = 0; h < S / 2; ++h) {
      const int j = 2 * h;
      out[h] = make_double2(in[j], j + 1 < n ? in[j + 1] : 0.0);
    }
  }
}

__global__ void k_dense_fill(uint32_t* __restrict__ table, int64_t size) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < size;
       i += (int64_t)gridDim.x * blockDim.x)
    table[i] = 0xFFFFFFFFu;
}

__global__ void k_dense_scatter(const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                                uint32_t* __restrict__ table) {
  const uint32_t M = *d_M;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < M;
       c += (int64_t)gridDim.x * blockDim.x)
    table[cell_key[c]] = (uint32_t)c;
}

// Z-order level: the row-major cell index (strides of the level) of each
// cell, -> its position in the cell table.  The table is not cleared first:
// a reader checks that an entry names a cell of the level with its key.
template <int DIM>
__global__ void k_dense_scatter_z(const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                                  GeomDev gd, uint32_t* __restrict__ table) {
  const uint32_t M = *d_M;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < M;
       c += (int64_t)gridDim.x * blockDim.x) {
    int64_t cc[DIM];
    zorder_coords<DIM>(cell_key[c], gd.zbits, cc);
    uint64_t rk = 0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) rk += (uint64_t)cc[j] * gd.stride[j];
    table[rk] = (uint32_t)c;
  }
}

// Index of the first cell whose key is >= key (binary search in cell_key[0..M)).
__device__ inline uint32_t lower_bound_key(const uint64_t* __restrict__ cell_key, uint32_t lo,
                                           uint32_t hi, uint64_t key) {
  // short ranges (most grid rows): a linear probe, the loads independent
  if (hi - lo <= 4) {
    uint32_t f = hi;
    for (uint32_t i = hi; i > lo; --i)
      if (cell_key[i - 1] >= key) f = i - 1;
    return f;
  }
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (cell_key[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int DIM>
__device__ inline void range_of(int r, const int64_t (&cc)[DIM],
                                const uint32_t* __restrict__ cell_start,
                                const uint64_t* __restrict__ cell_key, uint32_t M,
                                const uint32_t* __restrict__ dense,
                                const uint2* __restrict__ rowtab, const struct GeomDev& gd,
                                uint32_t& start, uint32_t& mid0, uint32_t& mid1, uint32_t& end);

// A group of S lanes per cell (S = the power of two >= 3^(n-1), at most 64):
// lane l computes row segments r = l, l+S, ...; the non-empty ones are written
// compacted (in r order) with their slot r, their count and the cell's total
// candidate count.  The cell's coordinates are recomputed from its first
// point with the key formula, so no key decoding is needed.
template <int DIM>
__global__ void k_neighbor_ranges(const double* __restrict__ Xs, int64_t N,
                                  const uint32_t* __restrict__ cell_start,
                                  const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                                  const uint32_t* __restrict__ dense,
                                  const uint2* __restrict__ rowtab,
                                  const uint8_t* __restrict__ cell_active, uint8_t active_tag,
                                  GeomDev gd, uint32_t* __restrict__ ranges,
                                  uint8_t* __restrict__ rslot,
                                  uint32_t* __restrict__ nrng,
                                  uint32_t* __restrict__ cand_count) {
  constexpr int R = DIM == 2 ? 3 : DIM == 3 ? 9 : DIM == 4 ? 27 : DIM == 5 ? 81 : 243;
  constexpr int S = R <= 4 ? 4 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
  const uint32_t M = *d_M;
  const int lane = threadIdx.x & 63;
  const int l = lane % S;
  const int sub = lane / S;
  const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / S);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x / S) + threadIdx.x / S; c < (int64_t)M;
       c += groups) {
    if (cell_active && cell_active[c] != active_tag) continue;
    const uint32_t p0 = cell_start[c];
    int64_t cc[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      cc[j] = cell_coord(Xs[(int64_t)p0 * point_stride(DIM) + j], gd.lo[j], gd.inv_w);
    uint32_t count = 0, cand = 0;
    for (int rb = 0; rb < R; rb += S) {
      const int r = rb + l;
      uint32_t start = 0, mid0 = 0, mid1 = 0, end = 0;
      if (r < R)
        range_of<DIM>(r, cc, cell_start, cell_key, M, dense, rowtab, gd, start, mid0, mid1, end);
      const bool ne = end > start;
      const uint64_t m = (S == 64 ? __ballot(ne) : (__ballot(ne) >> (sub * S))) &
                         (S == 64 ? ~0ull : ((1ull << S) - 1ull));
      if (ne) {
        const uint32_t pos = count + (uint32_t)__popcll(m & lt);
        reinterpret_cast<uint4*>(ranges)[(int64_t)c * R + pos] = make_uint4(start, mid0, mid1, end);
        rslot[(int64_t)c * R + pos] = (uint8_t)r;
        cand += end - start;
      }
      count += (uint32_t)__popcll(m);
    }
    // the group's total into its lane 0 (S need not be a power of two)
    if constexpr ((S & (S - 1)) == 0) {
#pragma unroll
      for (int o = 1; o < S; o <<= 1) cand += __shfl_xor(cand, o, 64);
    } else {
      uint32_t tot = 0;
#pragma unroll
      for (int o = 0; o < S; ++o) tot += __shfl(cand, sub * S + o, 64);
      cand = tot;
    }
    if (l == 0) {
      nrng[c] = count;
      cand_count[c] = cand;
    }
  }
}

// Point range [start, end) of row segment r of the cell with coordinates cc
// (offsets o_0..o_{DIM-2} in {-1,0,1}, o_0 slowest; last coordinate within
// one of the cell's), split at mid0 and mid1: [start, mid0) holds the points
// whose last cell coordinate is below the cell's, [mid0, mid1) those equal to
// it, [mid1, end) those above.  Empty: all four 0.
template <int DIM>
__device__ inline void range_of(int r, const int64_t (&cc)[DIM],
                                const uint32_t* __restrict__ cell_start,
                                const uint64_t* __restrict__ cell_key, uint32_t M,
                                const uint32_t* __restrict__ dense,
                                const uint2* __restrict__ rowtab, const GeomDev& gd,
                                uint32_t& start, uint32_t& mid0, uint32_t& mid1, uint32_t& end) {
  {
    bool inside = true;
    uint64_t prefix = 0, row = 0;
    int rr = r;
    int64_t nb[DIM];
#pragma unroll
    for (int j = DIM - 2; j >= 0; --j) {
      int o = rr % 3 - 1;
      rr /= 3;
      nb[j] = cc[j] + o;
      if (nb[j] < 0 || nb[j] >= gd.g[j]) inside = false;
    }
    start = 0;
    end = 0;
    mid0 = 0;
    mid1 = 0;
    if (inside) {
#pragma unroll
      for (int j = 0; j < DIM - 1; ++j) {
        prefix += (uint64_t)nb[j] * gd.stride[j];
        row += (uint64_t)nb[j] * gd.rstride[j];  // prefix / g_last without a division
      }
      const int64_t last = cc[DIM - 1];
      const int64_t a = last > 0 ? last - 1 : 0;
      const int64_t b = last + 1 < gd.g[DIM - 1] ? last + 1 : gd.g[DIM - 1] - 1;
      // the segment's cells are consecutive in sorted order; the first one
      // with t >= last starts the middle part, the first with t > last the
      // upper part
      uint32_t c_lo = 0xFFFFFFFFu, c_hi = 0xFFFFFFFFu;  // first / last cell of the segment
      uint32_t c_mid = 0xFFFFFFFFu, c_up = 0xFFFFFFFFu;
      if (dense) {
        for (int64_t t = a; t <= b; ++t) {
          uint32_t ci = dense[prefix + (uint64_t)t];
          if (ci != 0xFFFFFFFFu) {
            if (c_lo == 0xFFFFFFFFu) c_lo = ci;
            c_hi = ci;
            if (t >= last && c_mid == 0xFFFFFFFFu) c_mid = ci;
            if (t > last && c_up == 0xFFFFFFFFu) c_up = ci;
          }
        }
      } else {
        const uint64_t klo = prefix + (uint64_t)a, khi = prefix + (uint64_t)b;
        const uint64_t kmid = prefix + (uint64_t)last;
        // cells of the row (a CSR row table when there is one, else all)
        uint32_t rs = 0, re = M;
        if (rowtab) {
          const uint2 rr2 = rowtab[row];
          rs = rr2.x;
          re = rr2.y;
        }
        uint32_t f = lower_bound_key(cell_key, rs, re, klo);
        for (uint32_t l = f; l < re && cell_key[l] <= khi; ++l) {
          const uint64_t k = cell_key[l];
          if (c_lo == 0xFFFFFFFFu) c_lo = l;
          c_hi = l;
          if (k >= kmid && c_mid == 0xFFFFFFFFu) c_mid = l;
          if (k > kmid && c_up == 0xFFFFFFFFu) c_up = l;
        }
      }
      if (c_lo != 0xFFFFFFFFu) {
        start = cell_start[c_lo];
        end = cell_start[c_hi + 1];
        mid0 = c_mid != 0xFFFFFFFFu ? cell_start[c_mid] : end;
        mid1 = c_up != 0xFFFFFFFFu ? cell_start[c_up] : end;
      }
    }
  }
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_item_keys(const int32_t* __restrict__ active, int64_t n_active, int G,
                            const uint32_t* __restrict__ cell_of,
                            const uint32_t* __restrict__ cand_count, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ vals, int64_t n_items) {
  for (int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; it < n_items;
       it += (int64_t)gridDim.x * blockDim.x) {
    uint64_t est = 0;
    int64_t s0 = it * G, s1 = s0 + G < n_active ? s0 + G : n_active;
    for (int64_t s = s0; s < s1; ++s) {
      int64_t q = active ? active[s] : s;
      est += cand_count[cell_of[q]];
    }
    // density class: half-octaves of the estimate, densest class first; the
    // stable sort keeps cell order (spatial locality) inside a class
    const int cls = est ? (int)(2.0 * log2((double)est)) : 0;
    const uint64_t chunk = (uint64_t)(it * kXcds / n_items);
    keys[it] = (chunk << 6) | (uint64_t)(63 - (cls > 63 ? 63 : cls));
    vals[it] = (int32_t)it;
  }
}

__global__ void k_active_cand_sum(const int32_t* __restrict__ active, int64_t n_active,
                                  const uint32_t* __restrict__ cell_of,
                                  const uint32_t* __restrict__ cand_count, uint64_t* sum) {
  __shared__ unsigned long long red[kBlock];
  __shared__ unsigned int redm[kBlock];
  unsigned long long s = 0;
  unsigned int m = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_active;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t q = active ? active[i] : i;
    const unsigned int c = cand_count[cell_of[q]];
    s += c;
    m = max(m, c);
  }
  red[threadIdx.x] = s;
  redm[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[threadIdx.x] += red[threadIdx.x + w];
      redm[threadIdx.x] = max(redm[threadIdx.x], redm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long*)sum, red[0]);
    atomicMax((unsigned long long*)(sum + 1), (unsigned long long)redm[0]);
  }
}

// Active queries (sorted positions) whose cell has at least heavy_min
// candidates, appended to list (one atomic per wavefront); *count ends at
// their number.
__global__ void k_heavy_list(const int32_t* __restrict__ active, int64_t n_active,
                             const uint32_t* __restrict__ cell_of,
                             const uint32_t* __restrict__ cand_count, uint32_t heavy_min,
                             int32_t* __restrict__ list, int32_t* count,
                             unsigned long long* cand_sum) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < n_active;
       base += stride) {
    const int64_t i = base + lane;
    int32_t q = 0;
    bool h = false;
    unsigned long long cs = 0;
    if (i < n_active) {
      q = active ? active[i] : (int32_t)i;
      const uint32_t cq = cand_count[cell_of[q]];
      h = cq >= heavy_min;
      cs = h ? cq : 0ull;
    }
    const uint64_t m = __ballot(h);
    if (m) {
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) cs += __shfl_xor(cs, o, 64);
      int b = 0;
      if (lane == 0) {
        b = atomicAdd(count, (int)__popcll(m));
        atomicAdd(cand_sum, cs);
      }
      b = __shfl(b, 0, 64);
      const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
      if (h) list[b + (int)__popcll(m & lt)] = q;
    }
  }
}

__global__ void k_mark_failed(const int32_t* __restrict__ fail_list, const int32_t* d_count,
                              uint8_t* __restrict__ failed, uint8_t tag) {
  const int64_t cnt = *d_count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x)
    failed[fail_list[i]] = tag;
}

__global__ void k_pos_to_id(int32_t* __restrict__ list, int64_t n,
                            const int32_t* __restrict__ perm) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    list[i] = perm[list[i]];
}

// Position of the cell with key k in cell_key[0..M) (sorted, distinct keys),
// searched outward from position c0 (key k0) by galloping, then bisection;
// 0xFFFFFFFF when no cell has that key.
__device__ inline uint32_t find_cell_near(const uint64_t* __restrict__ ck, uint32_t M, uint32_t c0,
                                          uint64_t k0, uint64_t k) {
  if (k == k0) return c0;
  uint64_t lo, hi;  // the first position with key >= k lies in [lo, hi]
  if (k > k0) {
    uint64_t prev = c0, step = 1;
    for (;;) {
      const uint64_t probe = (uint64_t)c0 + step;
      if (probe >= M) {
        hi = M;
        break;
      }
      if (ck[probe] >= k) {
        hi = probe;
        break;
      }
      prev = probe;
      step <<= 1;
    }
    lo = prev + 1;
  } else {
    uint64_t prev = c0, step = 1;  // ck[prev] >= k
    for (;;) {
      if (step > c0) {
        lo = 0;
        break;
      }
      const uint64_t probe = (uint64_t)c0 - step;
      if (ck[probe] < k) {
        lo = probe + 1;
        break;
      }
      prev = probe;
      step <<= 1;
    }
    hi = prev;
  }
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (ck[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < M && ck[lo] == k) ? (uint32_t)lo : 0xFFFFFFFFu;
}

// Z-order level ranges: a group of S lanes per (flagged) cell, lane l taking
// the block cells r = l, l + S, ... (r in [0, 3^DIM), offsets in base 3, the
// last dimension fastest); the non-empty ones are written compacted in r
// order as described in kernels.hpp.
template <int DIM>
__global__ void k_neighbor_ranges_z(const uint32_t* __restrict__ cell_start,
                                    const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                                    const uint8_t* __restrict__ cell_active, uint8_t active_tag,
                                    const uint32_t* __restrict__ dense,
                                    GeomDev gd, uint32_t* __restrict__ ranges,
                                    uint8_t* __restrict__ rslot, uint32_t* __restrict__ nrng,
                                    uint32_t* __restrict__ cand_count) {
  constexpr int R = DIM == 2 ? 9 : DIM == 3 ? 27 : 81;
  // lanes per cell: one per neighbour up to a wavefront (2-D: 7 cells of 9
  // lanes per wavefront, the last lane idle)
  constexpr int S = R <= 64 ? R : 64;
  constexpr int GPW = 64 / S;  // cells per wavefront
  const uint32_t M = *d_M;
  const int lane = threadIdx.x & 63;
  const int l = lane % S;
  const int sub = lane / S;
  const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
  const uint64_t gmask = S >= 64 ? ~0ull : ((1ull << (S & 63)) - 1ull);
  const int64_t wpb = blockDim.x / 64;
  const int64_t groups = (int64_t)gridDim.x * wpb * GPW;
  const int64_t c0 = sub < GPW ? ((int64_t)blockIdx.x * wpb + threadIdx.x / 64) * GPW + sub
                               : (int64_t)M;  // the idle lane takes no cell
  for (int64_t c = c0; c < (int64_t)M; c += groups) {
    if (cell_active && cell_active[c] != active_tag) continue;
    const uint64_t k0 = cell_key[c];
    int64_t cc[DIM];
    zorder_coords<DIM>(k0, gd.zbits, cc);
    uint32_t count = 0, cand = 0;
    for (int rb = 0; rb < R; rb += S) {
      const int r = rb + l;
      uint32_t start = 0, end = 0;
      int olast = 0;
      if (r < R) {
        int64_t nb[DIM];
        bool inside = true;
        int rr = r;
#pragma unroll
        for (int j = DIM - 1; j >= 0; --j) {
          const int o = rr % 3 - 1;
          rr /= 3;
          if (j == DIM - 1) olast = o;
          nb[j] = cc[j] + o;
          if (nb[j] < 0 || nb[j] >= gd.g[j]) inside = false;
        }
        if (inside) {
          const uint64_t nk = zorder_key<DIM>(nb, gd.zbits);
          uint32_t f;
          if (dense) {
            // the level's cell at these coordinates, if the entry is this
            // level's: entries are never cleared, so one is trusted only
            // when it names a cell of the level with this key
            uint64_t rk = 0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) rk += (uint64_t)nb[j] * gd.stride[j];
            f = dense[rk];
            if (f >= M || cell_key[f] != nk) f = 0xFFFFFFFFu;
          } else {
            f = find_cell_near(cell_key, M, (uint32_t)c, k0, nk);
          }
          if (f != 0xFFFFFFFFu) {
            start = cell_start[f];
            end = cell_start[f + 1];
          }
        }
      }
      const bool ne = end > start;
      const uint64_t m = (S == 64 ? __ballot(ne) : (__ballot(ne) >> (sub * S))) & gmask;
      if (ne) {
        const uint32_t pos = count + (uint32_t)__popcll(m & lt);
        const uint32_t m0 = olast < 0 ? end : start;   // the cell is the lower part,
        const uint32_t m1 = olast > 0 ? start : end;   // the middle or the upper part
        reinterpret_cast<uint4*>(ranges)[(int64_t)c * R + pos] = make_uint4(start, m0, m1, end);
        rslot[(int64_t)c * R + pos] = (uint8_t)(r / 3);
        cand += end - start;
      }
      count += (uint32_t)__popcll(m);
    }
    // the group's total into its lane 0 (S need not be a power of two)
    if constexpr ((S & (S - 1)) == 0) {
#pragma unroll
      for (int o = 1; o < S; o <<= 1) cand += __shfl_xor(cand, o, 64);
    } else {
      uint32_t tot = 0;
#pragma unroll
      for (int o = 0; o < S; ++o) tot += __shfl(cand, sub * S + o, 64);
      cand = tot;
    }
    if (l == 0) {
      nrng[c] = count;
      cand_count[c] = cand;
    }
  }
}

// First position in keys[0..N) whose key is >= k (N if none).
template <class KeyT>
__device__ inline int64_t lower_bound_key(const KeyT* __restrict__ keys, int64_t N, uint64_t k) {
  int64_t lo = 0, hi = N;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)keys[mid] < k)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// A Z-order level with few active queries, without its cell table: slot i
// holds the ranges of the 3^n block of the i-th active query (sorted
// position q), each neighbour cell's points found in the sorted level-0
// keys as the run whose keys shifted right by zshift equal the cell's key
// (two binary searches), in the format of k_neighbor_ranges_z; cell_of[q] =
// i, and *d_M = the number of slots.  A group of S lanes per query.
template <int DIM, class KeyT>
__global__ void k_sparse_ranges_z(const KeyT* __restrict__ keys, int64_t N,
                                  const int32_t* __restrict__ active, int64_t n_active,
                                  const uint32_t* n_dev, int zshift, GeomDev gd,
                                  uint32_t* __restrict__ ranges, uint8_t* __restrict__ rslot,
                                  uint32_t* __restrict__ nrng, uint32_t* __restrict__ cand_count,
                                  uint32_t* __restrict__ cell_of, uint32_t* __restrict__ d_M) {
  constexpr int R = DIM == 2 ? 9 : DIM == 3 ? 27 : 81;
  constexpr int S = R <= 64 ? R : 64;
  constexpr int GPW = 64 / S;
  const int64_t na = n_dev ? min(n_active, (int64_t)*n_dev) : n_active;
  if (blockIdx.x == 0 && threadIdx.x == 0) *d_M = (uint32_t)na;
  const int lane = threadIdx.x & 63;
  const int l = lane % S;
  const int sub = lane / S;
  const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
  const uint64_t gmask = S >= 64 ? ~0ull : ((1ull << (S & 63)) - 1ull);
  const int64_t wpb = blockDim.x / 64;
  const int64_t groups = (int64_t)gridDim.x * wpb * GPW;
  const int64_t i0 = sub < GPW ? ((int64_t)blockIdx.x * wpb + threadIdx.x / 64) * GPW + sub : na;
  for (int64_t i = i0; i < na; i += groups) {
    const int32_t q = active[i];
    const uint64_t k0 = (uint64_t)keys[q] >> zshift;
    int64_t cc[DIM];
    zorder_coords<DIM>(k0, gd.zbits, cc);
    uint32_t count = 0, cand = 0;
    for (int rb = 0; rb < R; rb += S) {
      const int r = rb + l;
      uint32_t start = 0, end = 0;
      int olast = 0;
      if (r < R) {
        int64_t nb[DIM];
        bool inside = true;
        int rr = r;
#pragma unroll
        for (int j = DIM - 1; j >= 0; --j) {
          const int o = rr % 3 - 1;
          rr /= 3;
          if (j == DIM - 1) olast = o;
          nb[j] = cc[j] + o;
          if (nb[j] < 0 || nb[j] >= gd.g[j]) inside = false;
        }
        if (inside) {
          const uint64_t nk = zorder_key<DIM>(nb, gd.zbits);
          start = (uint32_t)lower_bound_key(keys, N, nk << zshift);
          end = (uint32_t)lower_bound_key(keys, N, (nk + 1) << zshift);
        }
      }
      const bool ne = end > start;
      const uint64_t m = (S == 64 ? __ballot(ne) : (__ballot(ne) >> (sub * S))) & gmask;
      if (ne) {
        const uint32_t pos = count + (uint32_t)__popcll(m & lt);
        const uint32_t m0 = olast < 0 ? end : start;
        const uint32_t m1 = olast > 0 ? start : end;
        reinterpret_cast<uint4*>(ranges)[i * R + pos] = make_uint4(start, m0, m1, end);
        rslot[i * R + pos] = (uint8_t)(r / 3);
        cand += end - start;
      }
      count += (uint32_t)__popcll(m);
    }
    if constexpr ((S & (S - 1)) == 0) {
#pragma unroll
      for (int o = 1; o < S; o <<= 1) cand += __shfl_xor(cand, o, 64);
    } else {
      uint32_t tot = 0;
#pragma unroll
      for (int o = 0; o < S; ++o) tot += __shfl(cand, sub * S + o, 64);
      cand = tot;
    }
    if (l == 0) {
      nrng[i] = count;
      cand_count[i] = cand;
      cell_of[q] = (uint32_t)i;
    }
  }
}

// Index of the first cell whose key is >= key in cell_key[0..M) (M >= 1),
// clamped to M - 1: a starting point for the galloping search.
__device__ inline uint32_t start_cell(const uint64_t* __restrict__ cell_key, uint32_t M,
                                      uint64_t key) {
  uint32_t lo = 0, hi = M;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (cell_key[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < M ? lo : M - 1;
}

// Ranges of external queries (a join of a query set with the indexed set):
// a query need not lie in any non-empty cell, so it gets a slot of its own,
// slot i for the query at position base + i of the point array: its cell
// coordinates come from its coordinates, its block's ranges are looked up in
// the cell table (Z-order: galloping from the query key's place in it;
// row-major: the row-segment lookup), written to slot i in the cells'
// format, and cell_of[q] = i.  A group of S lanes per active query.
template <int DIM, bool ZL>
__global__ void k_query_ranges(const double* __restrict__ Xs, const int32_t* __restrict__ active,
                               int64_t n_active, const uint32_t* n_dev, int64_t base, int64_t nq,
                               const uint32_t* __restrict__ cell_start,
                               const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                               const uint32_t* __restrict__ dense,
                               const uint2* __restrict__ rowtab, GeomDev gd,
                               uint32_t* __restrict__ cell_of, uint32_t* __restrict__ ranges,
                               uint8_t* __restrict__ rslot, uint32_t* __restrict__ nrng,
                               uint32_t* __restrict__ cand_count) {
  constexpr int R = ZL ? (DIM == 2 ? 9 : DIM == 3 ? 27 : 81)
                       : (DIM == 2 ? 3 : DIM == 3 ? 9 : DIM == 4 ? 27 : DIM == 5 ? 81 : 243);
  constexpr int S = R <= 4 ? 4 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
  const uint32_t M = *d_M;
  const int lane = threadIdx.x & 63;
  const int l = lane % S;
  const int sub = lane / S;
  const uint64_t lt = l == 0 ? 0ull : (~0ull >> (64 - l));
  const int64_t groups = (int64_t)gridDim.x * (blockDim.x / S);
  const int64_t na = n_dev ? min(n_active, (int64_t)*n_dev) : n_active;
  for (int64_t a = (int64_t)blockIdx.x * (blockDim.x / S) + threadIdx.x / S; a < na;
       a += groups) {
    const int32_t q = active[a];
    const int64_t i = (int64_t)q - base;
    if (i < 0 || i >= nq) continue;  // not a query position (never in a valid list)
    int64_t cc[DIM];
#pragma unroll
    for (int j = 0; j < DIM; ++j)
      cc[j] = cell_coord(Xs[(int64_t)q * point_stride(DIM) + j], gd.lo[j], gd.inv_w);
    uint32_t c0 = 0;
    uint64_t k0 = 0;
    if constexpr (ZL) {
      c0 = start_cell(cell_key, M, zorder_key<DIM>(cc, gd.zbits));
      k0 = cell_key[c0];
    }
    uint32_t count = 0, cand = 0;
    for (int rb = 0; rb < R; rb += S) {
      const int r = rb + l;
      uint32_t start = 0, mid0 = 0, mid1 = 0, end = 0;
      int slot = 0;
      if (r < R) {
        if constexpr (ZL) {
          int64_t nb[DIM];
          bool inside = true;
          int rr = r, olast = 0;
#pragma unroll
          for (int j = DIM - 1; j >= 0; --j) {
            const int o = rr % 3 - 1;
            rr /= 3;
            if (j == DIM - 1) olast = o;
            nb[j] = cc[j] + o;
            if (nb[j] < 0 || nb[j] >= gd.g[j]) inside = false;
          }
          if (inside) {
            const uint32_t f = find_cell_near(cell_key, M, c0, k0, zorder_key<DIM>(nb, gd.zbits));
            if (f != 0xFFFFFFFFu) {
              start = cell_start[f];
              end = cell_start[f + 1];
            }
          }
          mid0 = olast < 0 ? end : start;
          mid1 = olast > 0 ? start : end;
          slot = r / 3;
        } else {
          range_of<DIM>(r, cc, cell_start, cell_key, M, dense, rowtab, gd, start, mid0, mid1,
                        end);
          slot = r;
        }
      }
      const bool ne = end > start;
      const uint64_t m = (S == 64 ? __ballot(ne) : (__ballot(ne) >> (sub * S))) &
                         (S == 64 ? ~0ull : ((1ull << S) - 1ull));
      if (ne) {
        const uint32_t pos = count + (uint32_t)__popcll(m & lt);
        reinterpret_cast<uint4*>(ranges)[i * R + pos] = make_uint4(start, mid0, mid1, end);
        rslot[i * R + pos] = (uint8_t)slot;
        cand += end - start;
      }
      count += (uint32_t)__popcll(m);
    }
#pragma unroll
    for (int o = 1; o < S; o <<= 1) cand += __shfl_xor(cand, o, 64);
    if (l == 0) {
      nrng[i] = count;
      cand_count[i] = cand;
      cell_of[q] = (uint32_t)i;
    }
  }
}

__global__ void k_iota(int32_t* __restrict__ out, int64_t n, int32_t base) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = base + (int32_t)i;
}


// Zero fill: `words` 32-bit words, then `tail` (< 4) trailing bytes.  A kernel
// rather than a memset node, so the join's launch sequence can be captured in
// a graph and replayed.
__global__ void k_zero(uint32_t* __restrict__ p, int64_t words, uint8_t* __restrict__ tailp,
                       int tail) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
  if (blockIdx.x == 0 && (int)threadIdx.x < tail) tailp[threadIdx.x] = 0;
}

int grid_for(int64_t n, int cap = 8192) {
  int64_t b = ceil_div(n, kBlock);
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

void launch_aos_to_soa(const double* D, int64_t N, int n, double* X, uint32_t* bad,
                       hipStream_t s) {
  k_aos_to_soa<<<grid_for(N * n), kBlock, 0, s>>>(D, N, n, X, bad);
  KNN_LAUNCHED();
}

void launch_bounds(const double* X, int64_t N, int n, double* part, double* lo, double* hi,
                   hipStream_t s) {
  int nb = grid_for(N, kBoundsBlocks);
  k_bounds_partial<<<nb, kBlock, 0, s>>>(X, N, n, part);
  KNN_LAUNCHED();
  k_bounds_final<<<1, kBlock, 0, s>>>(part, nb, n, lo, hi);
  KNN_LAUNCHED();
}

static size_t tile_area_elems(int64_t n) {
  // per tile of >= kLbMinTile elements: a count, and two 64-bit masks per
  // 64 elements (the deferral filter's keep and defer ballots)
  return (size_t)(ceil_div(n, kLbMinTile) + 1) * (2 + 4 * (kLbMinTile / 64)) + 16;
}

size_t scan_state_elems(int64_t n) {
  // scans of up to n elements, or of a radix histogram of n keys (the
  // look-back words), then the tile area of compactions of up to n elements
  const int64_t m = std::max<int64_t>(n, ((int64_t)1 << kMaxDigitBits) * ceil_div(n, kRadixTile));
  return 4 + 2 * (size_t)(ceil_div(m, kLbMinTile) + 1) + tile_area_elems(n);
}

uint32_t* scan_tile_area(uint32_t* state, int64_t state_elems, int64_t words) {
  // the last `words` (at most tile_area_elems of the size the state was made
  // for), 8-byte aligned: past every look-back word a scan of that size uses
  const int64_t start = (state_elems - words) & ~(int64_t)1;
  KNN_CHECK(words > 0 && start >= 64, KNN_EINTERNAL, "scan state too small for the tile area");
  return state + start;
}

void launch_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                           uint32_t* state, int64_t state_elems, hipStream_t s) {
  if (n <= 0) {
    if (total) launch_zero(total, sizeof(uint32_t), s);
    return;
  }
  const int64_t nb = ceil_div(n, kOneTile);
  KNN_CHECK(4 + 2 * nb <= state_elems, KNN_EINTERNAL, "scan state too small");
  const bool vec = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
  if (vec)
    k_scan_onepass<true><<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, nb, state, total);
  else
    k_scan_onepass<false><<<(unsigned)nb, kBlock, 0, s>>>(in, out, n, nb, state, total);
  KNN_LAUNCHED();
}

size_t radix_tmp_elems(int64_t n) {
  int64_t nb = ceil_div(n, kRadixTile);
  return (size_t)(((int64_t)1 << kMaxDigitBits) * nb);
}

template <class KeyT>
static bool radix_sort_pairs_t(KeyT* keys, int32_t* vals, KeyT* keys2, int32_t* vals2,
                               int64_t n, int bits, uint32_t* tmp, uint32_t* state,
                               int64_t state_elems, hipStream_t s) {
  if (n <= 1 || bits <= 0) return false;
  KNN_CHECK(bits <= (int)(8 * sizeof(KeyT)), KNN_EINTERNAL, "radix sort: more bits than the key");
  int64_t nb = ceil_div(n, kRadixTile);
  // 8-bit digits, scattered through LDS (coalesced digit runs); the direct
  // 11-bit scatter (one pass fewer, scattered stores) only for small sorts
  const bool lds = n >= 4 * kRadixTile;
  const int DB = lds ? 8 : ((bits + 10) / 11 < (bits + 7) / 8 ? 11 : 8);
  const int passes = (bits + DB - 1) / DB;
  const int64_t cnt = ((int64_t)1 << DB) * nb;
  uint32_t* hist = tmp;
  KeyT* src_k = keys;
  int32_t* src_v = vals;
  KeyT* dst_k = keys2;
  int32_t* dst_v = vals2;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = DB * ps;
    if (DB == 11)
      k_radix_hist<11, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(src_k, n, shift, hist, nb);
    else
      k_radix_hist<8, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(src_k, n, shift, hist, nb);
    KNN_LAUNCHED();
    launch_exclusive_scan(hist, hist, cnt, nullptr, state, state_elems, s);
    if (lds)
      k_radix_scatter_lds<KeyT><<<(unsigned)nb, kBlock, 0, s>>>(src_k, src_v, n, shift, hist, nb,
                                                                dst_k, dst_v);
    else if (DB == 11)
      k_radix_scatter<11, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(src_k, src_v, n, shift, hist, nb,
                                                                dst_k, dst_v);
    else
      k_radix_scatter<8, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(src_k, src_v, n, shift, hist, nb,
                                                               dst_k, dst_v);
    KNN_LAUNCHED();
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  return src_k != keys;
}

bool radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys2, int32_t* vals2,
                      int64_t n, int bits, uint32_t* tmp, uint32_t* state, int64_t state_elems,
                      hipStream_t s) {
  return radix_sort_pairs_t(keys, vals, keys2, vals2, n, bits, tmp, state, state_elems, s);
}

bool radix_sort_pairs(uint32_t* keys, int32_t* vals, uint32_t* keys2, int32_t* vals2,
                      int64_t n, int bits, uint32_t* tmp, uint32_t* state, int64_t state_elems,
                      hipStream_t s) {
  return radix_sort_pairs_t(keys, vals, keys2, vals2, n, bits, tmp, state, state_elems, s);
}

template <class KeyT>
static void launch_cell_keys_t(const double* X, int64_t N, const GridGeom& gg, KeyT* keys,
                               int32_t* vals, hipStream_t s) {
  KNN_CHECK(gg.key_bits <= (int)(8 * sizeof(KeyT)), KNN_EINTERNAL,
            "cell keys: more bits than the key");
  GeomDev gd = to_dev(gg);
  int nb = grid_for(N);
  switch (gg.dims) {
    case 2: k_cell_keys<2, KeyT><<<nb, kBlock, 0, s>>>(X, N, gd, keys, vals); break;
    case 3: k_cell_keys<3, KeyT><<<nb, kBlock, 0, s>>>(X, N, gd, keys, vals); break;
    case 4: k_cell_keys<4, KeyT><<<nb, kBlock, 0, s>>>(X, N, gd, keys, vals); break;
    case 5: k_cell_keys<5, KeyT><<<nb, kBlock, 0, s>>>(X, N, gd, keys, vals); break;
    case 6: k_cell_keys<6, KeyT><<<nb, kBlock, 0, s>>>(X, N, gd, keys, vals); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
}

void launch_cell_keys(const double* X, int64_t N, const GridGeom& gg, uint64_t* keys,
                      int32_t* vals, hipStream_t s) {
  launch_cell_keys_t(X, N, gg, keys, vals, s);
}

void launch_cell_keys(const double* X, int64_t N, const GridGeom& gg, uint32_t* keys,
                      int32_t* vals, hipStream_t s) {
  launch_cell_keys_t(X, N, gg, keys, vals, s);
}

void launch_cell_keys_points(const double* Xs, int64_t N, const GridGeom& gg, uint64_t* keys,
                             int32_t* vals, hipStream_t s) {
  GeomDev gd = to_dev(gg);
  int nb = grid_for(N);
  switch (gg.dims) {
    case 2: k_cell_keys_points<2><<<nb, kBlock, 0, s>>>(Xs, N, gd, keys, vals); break;
    case 3: k_cell_keys_points<3><<<nb, kBlock, 0, s>>>(Xs, N, gd, keys, vals); break;
    case 4: k_cell_keys_points<4><<<nb, kBlock, 0, s>>>(Xs, N, gd, keys, vals); break;
    case 5: k_cell_keys_points<5><<<nb, kBlock, 0, s>>>(Xs, N, gd, keys, vals); break;
    case 6: k_cell_keys_points<6><<<nb, kBlock, 0, s>>>(Xs, N, gd, keys, vals); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
}

void launch_gather_prev(const double* Xs_prev, const int32_t* perm_prev, const int32_t* pos,
                        int64_t N, int n, double* Xs, int32_t* perm, hipStream_t s) {
  k_gather_prev<<<grid_for(N), kBlock, 0, s>>>(Xs_prev, perm_prev, pos, N, point_stride(n), Xs,
                                               perm);
  KNN_LAUNCHED();
}

template <class KeyT>
static void build_cell_table_t(const KeyT* sorted_keys, int64_t N, uint32_t* cell_of,
                               uint64_t* cell_key, uint32_t* cell_start, uint32_t* d_M,
                               uint32_t* state, int64_t state_elems, hipStream_t s, int shift) {
  if (N <= 0) {
    launch_zero(d_M, sizeof(uint32_t), s);
    return;
  }
  const int64_t nb = ceil_div(N, kCtTile);
  KNN_CHECK(shift >= 0 && shift < 64, KNN_EINTERNAL, "cell table: key shift out of range");
  uint32_t* tw = scan_tile_area(state, state_elems, nb + 2);
  k_cell_table<false, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(sorted_keys, N, shift, cell_of,
                                                            cell_key, cell_start, d_M, tw);
  KNN_LAUNCHED();
  launch_exclusive_scan(tw, tw, nb, nullptr, state, state_elems, s);
  k_cell_table<true, KeyT><<<(unsigned)nb, kBlock, 0, s>>>(sorted_keys, N, shift, cell_of,
                                                           cell_key, cell_start, d_M, tw);
  KNN_LAUNCHED();
}

void build_cell_table(const uint64_t* sorted_keys, int64_t N, uint32_t* flags, uint32_t* cell_of,
                      uint64_t* cell_key, uint32_t* cell_start, uint32_t* d_M, uint32_t* state,
                      int64_t state_elems, hipStream_t s, int shift) {
  (void)flags;
  build_cell_table_t(sorted_keys, N, cell_of, cell_key, cell_start, d_M, state, state_elems, s,
                     shift);
}

void build_cell_table(const uint32_t* sorted_keys, int64_t N, uint32_t* flags, uint32_t* cell_of,
                      uint64_t* cell_key, uint32_t* cell_start, uint32_t* d_M, uint32_t* state,
                      int64_t state_elems, hipStream_t s, int shift) {
  (void)flags;
  build_cell_table_t(sorted_keys, N, cell_of, cell_key, cell_start, d_M, state, state_elems, s,
                     shift);
}

void launch_pos_to_id(int32_t* list, int64_t n, const int32_t* perm, hipStream_t s) {
  if (n <= 0) return;
  k_pos_to_id<<<grid_for(n), kBlock, 0, s>>>(list, n, perm);
  KNN_LAUNCHED();
}

void launch_neighbor_ranges_z(const uint32_t* cell_start, const uint64_t* cell_key,
                              const uint32_t* d_M, int64_t N, const uint8_t* cell_active,
                              uint8_t active_tag, const GridGeom& gg, uint32_t* dense,
                              int64_t dense_size, uint32_t* ranges, uint8_t* rslot,
                              uint32_t* nrng, uint32_t* cand_count, hipStream_t s) {
  KNN_CHECK(gg.zbits >= 0 && gg.dims <= kZMaxDims, KNN_EINTERNAL, "not a Z-order level");
  GeomDev gd = to_dev(gg);
  if (dense) {
    long double cells = 1;
    for (int j = 0; j < gg.dims; ++j) cells *= (long double)gg.g[j];
    KNN_CHECK(cells <= (long double)dense_size, KNN_EINTERNAL, "dense cell table too small");
    const int sb = grid_for(N);
    switch (gg.dims) {
      case 2: k_dense_scatter_z<2><<<sb, kBlock, 0, s>>>(cell_key, d_M, gd, dense); break;
      case 3: k_dense_scatter_z<3><<<sb, kBlock, 0, s>>>(cell_key, d_M, gd, dense); break;
      case 4: k_dense_scatter_z<4><<<sb, kBlock, 0, s>>>(cell_key, d_M, gd, dense); break;
      default: throw Error(KNN_EINVAL, "Z-order levels take 2-4 dimensions");
    }
    KNN_LAUNCHED();
  }
  const int S = gg.dims == 2 ? 9 : gg.dims == 3 ? 27 : 64;
  const int nb = grid_for(N * 64 / (64 / S), 65536);
  switch (gg.dims) {
    case 2: k_neighbor_ranges_z<2><<<nb, kBlock, 0, s>>>(cell_start, cell_key, d_M, cell_active, active_tag, dense, gd, ranges, rslot, nrng, cand_count); break;
    case 3: k_neighbor_ranges_z<3><<<nb, kBlock, 0, s>>>(cell_start, cell_key, d_M, cell_active, active_tag, dense, gd, ranges, rslot, nrng, cand_count); break;
    case 4: k_neighbor_ranges_z<4><<<nb, kBlock, 0, s>>>(cell_start, cell_key, d_M, cell_active, active_tag, dense, gd, ranges, rslot, nrng, cand_count); break;
    default: throw Error(KNN_EINVAL, "Z-order levels take 2-4 dimensions");
  }
  KNN_LAUNCHED();
}

template <class KeyT>
static void launch_sparse_ranges_z_t(const KeyT* sorted_keys, int64_t N, const int32_t* active,
                                     int64_t n_active, const uint32_t* n_dev, const GridGeom& gg,
                                     uint32_t* ranges, uint8_t* rslot, uint32_t* nrng,
                                     uint32_t* cand_count, uint32_t* cell_of, uint32_t* d_M,
                                     hipStream_t s) {
  KNN_CHECK(gg.zbits >= 0 && gg.dims <= kZMaxDims, KNN_EINTERNAL, "not a Z-order level");
  KNN_CHECK(gg.zshift >= 0 && gg.zshift + gg.dims * gg.zbits <= 62, KNN_EINTERNAL,
            "Z-order level: key bits out of range");
  if (n_active <= 0) {
    launch_zero(d_M, sizeof(uint32_t), s);
    return;
  }
  GeomDev gd = to_dev(gg);
  const int S = gg.dims == 2 ? 9 : gg.dims == 3 ? 27 : 64;
  const int nb = grid_for(ceil_div(n_active, 64 / S) * 64, 65536);
  switch (gg.dims) {
    case 2: k_sparse_ranges_z<2, KeyT><<<nb, kBlock, 0, s>>>(sorted_keys, N, active, n_active, n_dev, gg.zshift, gd, ranges, rslot, nrng, cand_count, cell_of, d_M); break;
    case 3: k_sparse_ranges_z<3, KeyT><<<nb, kBlock, 0, s>>>(sorted_keys, N, active, n_active, n_dev, gg.zshift, gd, ranges, rslot, nrng, cand_count, cell_of, d_M); break;
    case 4: k_sparse_ranges_z<4, KeyT><<<nb, kBlock, 0, s>>>(sorted_keys, N, active, n_active, n_dev, gg.zshift, gd, ranges, rslot, nrng, cand_count, cell_of, d_M); break;
    default: throw Error(KNN_EINVAL, "Z-order levels take 2-4 dimensions");
  }
  KNN_LAUNCHED();
}

void launch_sparse_ranges_z(const uint64_t* sorted_keys, int64_t N, const int32_t* active,
                            int64_t n_active, const uint32_t* n_dev, const GridGeom& gg,
                            uint32_t* ranges, uint8_t* rslot, uint32_t* nrng,
                            uint32_t* cand_count, uint32_t* cell_of, uint32_t* d_M,
                            hipStream_t s) {
  launch_sparse_ranges_z_t(sorted_keys, N, active, n_active, n_dev, gg, ranges, rslot, nrng,
                           cand_count, cell_of, d_M, s);
}

void launch_sparse_ranges_z(const uint32_t* sorted_keys, int64_t N, const int32_t* active,
                            int64_t n_active, const uint32_t* n_dev, const GridGeom& gg,
                            uint32_t* ranges, uint8_t* rslot, uint32_t* nrng,
                            uint32_t* cand_count, uint32_t* cell_of, uint32_t* d_M,
                            hipStream_t s) {
  launch_sparse_ranges_z_t(sorted_keys, N, active, n_active, n_dev, gg, ranges, rslot, nrng,
                           cand_count, cell_of, d_M, s);
}

void launch_active_list(const uint8_t* failed, uint8_t tag, const int32_t* perm, int64_t N,
                        int32_t* out, uint32_t* count, uint32_t* state, int64_t state_elems,
                        hipStream_t s, bool at_least, int32_t base) {
  if (N <= 0) {
    launch_zero(count, sizeof(uint32_t), s);
    return;
  }
  const int64_t nb = ceil_div(N, kCtTile);
  uint32_t* tw = scan_tile_area(state, state_elems, nb + 2);
  k_active_list<false><<<(unsigned)nb, kBlock, 0, s>>>(failed, tag, at_least, perm, N, base, out,
                                                       tw);
  KNN_LAUNCHED();
  launch_exclusive_scan(tw, tw, nb, count, state, state_elems, s);
  k_active_list<true><<<(unsigned)nb, kBlock, 0, s>>>(failed, tag, at_least, perm, N, base, out,
                                                      tw);
  KNN_LAUNCHED();
}

void launch_gather_points(const double* X, const int32_t* perm, int64_t N, int n, double* Xs,
                          hipStream_t s) {
  k_gather_points<<<grid_for(N), kBlock, 0, s>>>(X, perm, N, n, Xs);
  KNN_LAUNCHED();
}

__global__ void k_row_table(const uint64_t* __restrict__ cell_key, const uint32_t* d_M,
                            uint64_t g_last, uint2* __restrict__ rowtab) {
  const uint32_t M = *d_M;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < (int64_t)M;
       c += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t row = cell_key[c] / g_last;
    if (c == 0 || cell_key[c - 1] / g_last != row) rowtab[row].x = (uint32_t)c;
    if (c == (int64_t)M - 1 || cell_key[c + 1] / g_last != row) rowtab[row].y = (uint32_t)(c + 1);
  }
}

void launch_row_table(const uint64_t* cell_key, const uint32_t* d_M, int64_t N, uint64_t g_last,
                      uint2* rowtab, int64_t rows, hipStream_t s) {
  launch_zero(rowtab, (size_t)rows * sizeof(uint2), s);
  k_row_table<<<grid_for(N), kBlock, 0, s>>>(cell_key, d_M, g_last, rowtab);
  KNN_LAUNCHED();
}

void launch_dense_table(const uint64_t* cell_key, const uint32_t* d_M, int64_t N,
                        uint32_t* table, int64_t table_size, hipStream_t s) {
  k_dense_fill<<<grid_for(table_size), kBlock, 0, s>>>(table, table_size);
  KNN_LAUNCHED();
  k_dense_scatter<<<grid_for(N), kBlock, 0, s>>>(cell_key, d_M, table);
  KNN_LAUNCHED();
}

void launch_neighbor_ranges(const double* Xs, int64_t N, const uint32_t* cell_start,
                            const uint64_t* cell_key, const uint32_t* d_M,
                            const uint32_t* dense, const uint2* rowtab, const uint8_t* cell_active,
                            uint8_t active_tag, const GridGeom& gg, uint32_t* ranges,
                            uint8_t* rslot, uint32_t* nrng, uint32_t* cand_count, hipStream_t s) {
  GeomDev gd = to_dev(gg);
  const int S = gg.dims == 2 ? 4 : gg.dims == 3 ? 16 : gg.dims == 4 ? 32 : 64;
  const int nb = grid_for(N * S, 65536);
  switch (gg.dims) {
    case 2: k_neighbor_ranges<2><<<nb, kBlock, 0, s>>>(Xs, N, cell_start, cell_key, d_M, dense, rowtab, cell_active, active_tag, gd, ranges, rslot, nrng, cand_count); break;
    case 3: k_neighbor_ranges<3><<<nb, kBlock, 0, s>>>(Xs, N, cell_start, cell_key, d_M, dense, rowtab, cell_active, active_tag, gd, ranges, rslot, nrng, cand_count); break;
    case 4: k_neighbor_ranges<4><<<nb, kBlock, 0, s>>>(Xs, N, cell_start, cell_key, d_M, dense, rowtab, cell_active, active_tag, gd, ranges, rslot, nrng, cand_count); break;
    case 5: k_neighbor_ranges<5><<<nb, kBlock, 0, s>>>(Xs, N, cell_start, cell_key, d_M, dense, rowtab, cell_active, active_tag, gd, ranges, rslot, nrng, cand_count); break;
    case 6: k_neighbor_ranges<6><<<nb, kBlock, 0, s>>>(Xs, N, cell_start, cell_key, d_M, dense, rowtab, cell_active, active_tag, gd, ranges, rslot, nrng, cand_count); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
  KNN_LAUNCHED();
}

void launch_query_ranges(const double* Xs, const int32_t* active, int64_t n_active,
                         const uint32_t* n_dev, int64_t base, int64_t nq,
                         const uint32_t* cell_start, const uint64_t* cell_key,
                         const uint32_t* d_M, const uint32_t* dense, const uint2* rowtab,
                         const GridGeom& gg, bool zl, uint32_t* cell_of, uint32_t* ranges,
                         uint8_t* rslot, uint32_t* nrng, uint32_t* cand_count, hipStream_t s) {
  if (n_active <= 0) return;
  KNN_CHECK(!zl || gg.dims <= kZMaxDims, KNN_EINTERNAL, "Z-order levels take 2-4 dimensions");
  GeomDev gd = to_dev(gg);
  const int R = zl ? (gg.dims == 2 ? 9 : gg.dims == 3 ? 27 : 81)
                   : (gg.dims == 2 ? 3 : gg.dims == 3 ? 9 : gg.dims == 4 ? 27 : 81);
  const int S = R <= 4 ? 4 : R <= 16 ? 16 : R <= 32 ? 32 : 64;
  const int nb = grid_for(n_active * S, 65536);
#define KNN_QR(D, Z) k_query_ranges<D, Z><<<nb, kBlock, 0, s>>>(Xs, active, n_active, n_dev, base, nq, cell_start, cell_key, d_M, dense, rowtab, gd, cell_of, ranges, rslot, nrng, cand_count)
  if (zl) {
    switch (gg.dims) {
      case 2: KNN_QR(2, true); break;
      case 3: KNN_QR(3, true); break;
      case 4: KNN_QR(4, true); break;
      default: throw Error(KNN_EINVAL, "Z-order levels take 2-4 dimensions");
    }
  } else {
    switch (gg.dims) {
      case 2: KNN_QR(2, false); break;
      case 3: KNN_QR(3, false); break;
      case 4: KNN_QR(4, false); break;
      case 5: KNN_QR(5, false); break;
      case 6: KNN_QR(6, false); break;
      default: throw Error(KNN_EINVAL, "dims out of range");
    }
  }
#undef KNN_QR
  KNN_LAUNCHED();
}

void launch_iota(int32_t* out, int64_t n, int32_t base, hipStream_t s) {
  if (n <= 0) return;
  k_iota<<<grid_for(n), kBlock, 0, s>>>(out, n, base);
  KNN_LAUNCHED();
}

void launch_item_keys(const int32_t* active, int64_t n_active, int G, const uint32_t* cell_of,
                      const uint32_t* cand_count, uint64_t* keys, int32_t* vals, int64_t n_items,
                      hipStream_t s) {
  k_item_keys<<<grid_for(n_items), kBlock, 0, s>>>(active, n_active, G, cell_of, cand_count,
                                                    keys, vals, n_items);
  KNN_LAUNCHED();
}

void launch_active_cand_sum(const int32_t* active, int64_t n_active, const uint32_t* cell_of,
                            const uint32_t* cand_count, uint64_t* sum, hipStream_t s) {
  launch_zero(sum, 2 * sizeof(uint64_t), s);
  k_active_cand_sum<<<grid_for(n_active, 1024), kBlock, 0, s>>>(active, n_active, cell_of,
                                                                 cand_count, sum);
  KNN_LAUNCHED();
}

void launch_heavy_list(const int32_t* active, int64_t n_active, const uint32_t* cell_of,
                       const uint32_t* cand_count, uint32_t heavy_min, int32_t* list,
                       int32_t* count, unsigned long long* cand_sum, hipStream_t s) {
  k_heavy_list<<<grid_for(n_active, 2048), kBlock, 0, s>>>(active, n_active, cell_of, cand_count,
                                                            heavy_min, list, count, cand_sum);
  KNN_LAUNCHED();
}

void launch_mark_failed(const int32_t* fail_list, const int32_t* d_fail_count, int64_t max_fail,
                        uint8_t* failed, uint8_t tag, hipStream_t s) {
  k_mark_failed<<<grid_for(max_fail), kBlock, 0, s>>>(fail_list, d_fail_count, failed, tag);
  KNN_LAUNCHED();
}

__global__ void k_mark_cells_of(const int32_t* __restrict__ active, int64_t n_active,
                                const uint32_t* n_dev, const uint32_t* __restrict__ cell_of,
                                uint8_t* __restrict__ flags, uint8_t tag) {
  const int64_t n = n_dev ? min(n_active, (int64_t)*n_dev) : n_active;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[cell_of[active ? active[i] : (int32_t)i]] = tag;
}

void launch_mark_cells_of(const int32_t* active, int64_t n_active, const uint32_t* cell_of,
                          uint8_t* flags, uint8_t tag, hipStream_t s, const uint32_t* n_dev) {
  if (n_active <= 0) return;
  k_mark_cells_of<<<grid_for(n_active), kBlock, 0, s>>>(active, n_active, n_dev, cell_of, flags,
                                                        tag);
  KNN_LAUNCHED();
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  KNN_CHECK(((uintptr_t)p & 3) == 0, KNN_EINTERNAL, "zero fill needs a 4-byte aligned pointer");
  const int64_t words = (int64_t)(bytes / 4);
  const int tail = (int)(bytes % 4);
  k_zero<<<grid_for(std::max<int64_t>(words, 1)), kBlock, 0, s>>>(
      static_cast<uint32_t*>(p), words, static_cast<uint8_t*>(p) + words * 4, tail);
  KNN_LAUNCHED();
}

}  // namespace knn
