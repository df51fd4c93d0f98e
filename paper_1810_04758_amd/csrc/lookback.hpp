// lookback.hpp -- device helpers of the single-pass scans: block scans and the
// decoupled look-back over per-tile words.
//
// Tiles are taken in ticket order (an atomic counter), so every tile a block
// waits for belongs to a block that is already running.  A block publishes
// its tile's sum at once; then its first wavefront reads the words of
// kLookWords x 64 preceding tiles at a time (all loads in flight together),
// adds the sums up to the nearest inclusive prefix (or all of them, and goes
// on further back), and the block publishes its own inclusive prefix.
// State (uint32 array, zero-filled once when allocated, one stream's work at
// a time): [0..1] a 64-bit word, ticket (low half) and epoch (high half), so a
// block takes both in one atomic; [2] look-back errors; [4..] 64-bit tile
// words: flag (bit 63 inclusive prefix, bit 62 tile sum), epoch (bits 32..61),
// value (bits 0..31).  The epoch advances once per launch (the block with the
// last ticket moves it on and resets the ticket; the next launch on the
// stream starts after this one ends), so earlier words never need clearing.
// The words carry their values, so every access is a relaxed device-scope
// atomic (no cache write-back or invalidation).  A look-back that waits more
// than kLbSpinLimit rounds counts an error in state[2] and stops.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace knn {

constexpr uint64_t kLbFlagInc = 1ull << 63;
constexpr uint64_t kLbFlagAgg = 1ull << 62;
constexpr uint32_t kLbEpochMask = (1u << 30) - 1;
constexpr uint32_t kLbSpinLimit = 1u << 20;
constexpr int kLbLookWords = 4;

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread (blockDim == BLOCK); returns
// the exclusive prefix and writes the block total to *total.
template <int BLOCK>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[BLOCK / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BLOCK / 64; ++i) {
    if (i < w) base += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

struct LbTile {
  int64_t tile;
  uint32_t epoch;
};

// The block's tile and the launch's epoch (all threads; one barrier).
__device__ inline LbTile lb_take_tile(uint32_t* state, int64_t nb) {
  __shared__ uint32_t s_tile, s_epoch;
  unsigned long long* te = reinterpret_cast<unsigned long long*>(state);
  if (threadIdx.x == 0) {
    const unsigned long long old =
        __hip_atomic_fetch_add(te, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t t = (uint32_t)old;
    const uint32_t e = (uint32_t)(old >> 32) & kLbEpochMask;
    if ((int64_t)t == nb - 1)  // every ticket is taken: reset it, next epoch
      __hip_atomic_store(te, (unsigned long long)((e + 1) & kLbEpochMask) << 32,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_tile = t;
    s_epoch = e;
  }
  __syncthreads();
  return LbTile{(int64_t)s_tile, s_epoch};
}

// Publishes the tile's sum `agg` (thread 0's value counts), finds the sum of
// all earlier tiles and publishes the inclusive prefix; returns that sum in
// every thread (one barrier; s_excl: a __shared__ word of the caller).
__device__ inline uint32_t lb_tile_prefix(uint32_t* state, LbTile lt, uint32_t agg,
                                          uint32_t* s_excl) {
  unsigned long long* status = reinterpret_cast<unsigned long long*>(state + 4);
  const uint64_t etag = (uint64_t)lt.epoch << 32;
  if (threadIdx.x == 0)
    __hip_atomic_store(&status[lt.tile], (lt.tile == 0 ? kLbFlagInc : kLbFlagAgg) | etag | agg,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x < 64 && lt.tile > 0) {
    // predecessor j - (lane + 64 k) is word k of lane `lane`
    const int lane = threadIdx.x;
    uint32_t excl = 0;
    uint32_t spins = 0;
    int64_t j = lt.tile - 1;
    for (;;) {
      unsigned long long w[kLbLookWords];
#pragma unroll
      for (int k = 0; k < kLbLookWords; ++k) {
        const int64_t idx = j - lane - 64 * k;
        // before tile 0: an inclusive prefix of 0
        w[k] = idx >= 0 ? __hip_atomic_load(&status[idx], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                        : (kLbFlagInc | etag);
      }
      // nearest inclusive prefix: word kp, lane lp (kp = kLbLookWords: none)
      int kp = kLbLookWords, lp = 63;
      bool ready = true;
#pragma unroll
      for (int k = 0; k < kLbLookWords; ++k) {
        if (kp < kLbLookWords) break;
        const bool valid = (w[k] & (kLbFlagInc | kLbFlagAgg)) != 0 &&
                           (uint32_t)((w[k] >> 32) & kLbEpochMask) == lt.epoch;
        const uint64_t pm = __ballot(valid && (w[k] & kLbFlagInc) != 0);
        const uint64_t vm = __ballot(valid);
        const int last = pm ? __builtin_ctzll(pm) : 63;
        const uint64_t need = last == 63 ? ~0ull : ((2ull << last) - 1ull);
        if ((vm & need) != need) {
          ready = false;
          break;
        }
        if (pm) {
          kp = k;
          lp = last;
        }
      }
      if (!ready) {
        if (++spins > kLbSpinLimit) {
          if (lane == 0) atomicAdd(state + 2, 1u);
          break;
        }
        continue;
      }
      uint32_t part = 0;
#pragma unroll
      for (int k = 0; k < kLbLookWords; ++k)
        if (k < kp || (k == kp && lane <= lp)) part += (uint32_t)w[k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
      excl += part;
      if (kp < kLbLookWords) break;
      j -= 64 * kLbLookWords;
    }
    if (lane == 0) {
      __hip_atomic_store(&status[lt.tile], kLbFlagInc | etag | (uint32_t)(excl + agg),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *s_excl = excl;
    }
  } else if (threadIdx.x == 0) {
    *s_excl = 0;
  }
  __syncthreads();
  return *s_excl;
}

}  // namespace knn
