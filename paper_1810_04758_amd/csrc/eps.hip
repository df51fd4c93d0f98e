// eps.hip -- the two sampling kernels of the search-distance selection
// (Sec. 4.4): the mean distance between the points of a small sample
// (eps_mean), and the histogram of distances from sample points to every
// point of D, binned up to eps_mean.
#pragma clang fp contract(off)

#include <cmath>

#include "kernels.hpp"

namespace knn {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double sq_dist_soa(const double* __restrict__ X, int64_t N, int n,
                                              int64_t a, const double* qa) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) {
    double t = __dsub_rn(X[(int64_t)j * N + a], qa[j]);
    s = __dadd_rn(s, __dmul_rn(t, t));
  }
  return s;
}

// SX[j * ns + i] = X[j * N + sample[i]]: the sample's coordinates, compact
// (the pair loop then reads a few hundred KB instead of gathering from D).
__global__ void k_gather_sample(const double* __restrict__ X, int64_t N, int n,
                                const int64_t* __restrict__ sample, int64_t ns,
                                double* __restrict__ SX) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ns;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t id = sample[i];
    for (int j = 0; j < n; ++j) SX[(int64_t)j * ns + i] = X[(int64_t)j * N + id];
  }
}

// Block `a` sums the distances of sample point a to the sample points after it.
__global__ void k_pair_sums(const double* __restrict__ SX, int n, int64_t ns,
                            double* __restrict__ part) {
  __shared__ double red[kBlock];
  for (int64_t a = blockIdx.x; a < ns; a += gridDim.x) {
    double qa[kMaxDims];
    for (int j = 0; j < n; ++j) qa[j] = SX[(int64_t)j * ns + a];
    double s = 0.0;
    for (int64_t b = a + 1 + threadIdx.x; b < ns; b += blockDim.x)
      s += sqrt(sq_dist_soa(SX, ns, n, b, qa));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[a] = red[0];
    __syncthreads();
  }
}

constexpr int kSampleChunk = 256;
// points per thread in the distance histogram: 4 on a pass over every point
// (one LDS read of a sample point serves four pairs), 1 on a strided estimate
// pass (four times the workgroups: a few hundred workgroups of four points
// per thread left one wavefront per SIMD and no latency hidden)
constexpr int kPtsAll = 4;
constexpr int kMaxBins = 4096;

// Bin of a distance, floor(sqrt(d2) * inv_bw) with the correctly rounded
// square root.  A single-precision estimate (relative error below 2^-21:
// the conversion of d2, the hardware square root and two products) decides
// the bin unless it lies within 2^-18 (relative) of an integer; only then is
// the double-precision value taken.  That error bound holds only while every
// float involved is a normal number, so the estimate is used only for d2 in
// [2^-100, 2^100] and when inv_bw lies in [2^-60, 2^60] (use_f, checked once
// on the host): sqrt(d2) is then within [2^-50, 2^50] and the estimate within
// [2^-110, 2^110], far inside float's normal range.  Other values take the
// double-precision path.
__device__ __forceinline__ int dist_bin(double d2, double inv_bw, float inv_bw_f, bool use_f) {
  if (use_f && d2 >= 0x1p-100 && d2 <= 0x1p100) {
    const float t = __builtin_amdgcn_sqrtf((float)d2) * inv_bw_f;
    const float r = rintf(t);
    if (fabsf(t - r) > t * 0x1p-18f) return (int)floorf(t);
  }
  return (int)floor(sqrt(d2) * inv_bw);
}

// Each thread takes points p = i * pstride (every point when pstride = 1);
// the sample points of a chunk sit in LDS.  Only bins below count_bins are
// counted (pairs certainly beyond them skip the bin arithmetic).  The
// per-block histogram is accumulated in LDS (uint32) and added to the global
// uint64 counts at the end.
// skip_f: a single-precision squared distance above it proves the pair's
// double-precision d^2 above skip_d2 (see launch_dist_histogram), so most far
// pairs are rejected at single-precision rate; +inf disables the test.
template <int DIM, int kPts>
__global__ void k_dist_histogram(const double* __restrict__ X, int64_t N, int64_t pstride,
                                 const int64_t* __restrict__ sample, int64_t ns, double inv_bw,
                                 int count_bins, double skip_d2, float skip_f,
                                 uint64_t* __restrict__ counts) {
  const int n_bins = count_bins;
  __shared__ uint32_t h[kMaxBins];
  const float inv_bw_f = (float)inv_bw;
  const bool use_f = inv_bw >= 0x1p-60 && inv_bw <= 0x1p60;
  __shared__ double sx[DIM][kSampleChunk];
  __shared__ float sxf[DIM][kSampleChunk];
  __shared__ int64_t sid[kSampleChunk];
  for (int b = threadIdx.x; b < n_bins; b += blockDim.x) h[b] = 0;
  for (int64_t c0 = 0; c0 < ns; c0 += kSampleChunk) {
    const int cn = (int)((ns - c0) < kSampleChunk ? (ns - c0) : kSampleChunk);
    __syncthreads();
    for (int i = threadIdx.x; i < cn; i += blockDim.x) {
      int64_t id = sample[c0 + i];
      sid[i] = id;
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        sx[j][i] = X[(int64_t)j * N + id];
        sxf[j][i] = (float)sx[j][i];
      }
    }
    __syncthreads();
    // each thread takes kPts points (the LDS read of a sample point serves
    // all of them): point index t0 + u * blockDim (u < kPts), point p =
    // index * pstride
    const int64_t nP = (N + pstride - 1) / pstride;
    for (int64_t t0 = blockIdx.x * (int64_t)blockDim.x * kPts + threadIdx.x; t0 < nP;
         t0 += (int64_t)gridDim.x * blockDim.x * kPts) {
      double x[kPts][DIM];
      float xf[kPts][DIM];
      int64_t pp[kPts];
#pragma unroll
      for (int u = 0; u < kPts; ++u) {
        const int64_t t = t0 + (int64_t)u * blockDim.x;
        pp[u] = t < nP ? t * pstride : -1;
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
          x[u][j] = pp[u] >= 0 ? X[(int64_t)j * N + pp[u]] : 0.0;
          xf[u][j] = (float)x[u][j];
        }
      }
      for (int i = 0; i < cn; ++i) {
        float sq[DIM];
#pragma unroll
        for (int j = 0; j < DIM; ++j) sq[j] = sxf[j][i];
#pragma unroll
        for (int u = 0; u < kPts; ++u) {
          // each square added with one rounding (a fused multiply-add)
          float sf = 0.0f;
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            const float t = __fsub_rn(xf[u][j], sq[j]);
            sf = __builtin_fmaf(t, t, sf);
          }
          if (sf > skip_f) continue;  // provably beyond skip_d2
          if (pp[u] < 0) continue;
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            const double t = __dsub_rn(x[u][j], sx[j][i]);
            s = __dadd_rn(s, __dmul_rn(t, t));
          }
          if (s > skip_d2 || pp[u] == sid[i]) continue;  // beyond the last bin, or self
          const int b = dist_bin(s, inv_bw, inv_bw_f, use_f);
          if (b < n_bins) atomicAdd(&h[b], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
    if (h[b]) atomicAdd((unsigned long long*)&counts[b], (unsigned long long)h[b]);
}

}  // namespace

int launch_sample_pair_sums(const double* X, int64_t N, int n, const int64_t* sample,
                            int64_t ns, double* SX, double* part, hipStream_t s) {
  if (ns < 2) return 0;
  k_gather_sample<<<(int)std::min<int64_t>(ceil_div(ns, kBlock), 1024), kBlock, 0, s>>>(
      X, N, n, sample, ns, SX);
  KNN_LAUNCHED();
  int nb = (int)(ns < 65535 ? ns : 65535);
  k_pair_sums<<<nb, kBlock, 0, s>>>(SX, n, ns, part);
  KNN_LAUNCHED();
  return (int)ns;
}

void launch_dist_histogram(const double* X, int64_t N, int n, const int64_t* sample,
                           int64_t ns, double inv_bw, int n_bins, uint64_t* counts,
                           hipStream_t s, int count_bins, int64_t pstride, double max_abs) {
  KNN_CHECK(n_bins >= 1 && n_bins <= kMaxBins, KNN_EINVAL, "n_bins must be in [1, 4096]");
  if (count_bins <= 0 || count_bins > n_bins) count_bins = n_bins;
  KNN_CHECK(pstride >= 1, KNN_EINTERNAL, "histogram point stride must be >= 1");
  launch_zero(counts, n_bins * sizeof(uint64_t), s);
  if (ns <= 0 || N <= 0) return;
  // distances whose bin is certainly >= count_bins skip the square root
  double lim = (double)count_bins / inv_bw;
  double skip_d2 = lim * lim * 1.0001 + 1e-300;
  // The single-precision test.  With A = max_abs (every |coordinate|), each
  // coordinate's conversion to float errs by at most A 2^-24 (plus 2^-149
  // below float's normal range), so a float difference df_j of the converted
  // values satisfies |df_j| <= (|x_j - q_j| + e)(1 + 2^-24), e = 2 A 2^-24 +
  // 2^-148; the float sum sf of the n squares, each added by a fused
  // multiply-add (one rounding of 2^-24 per step), is at most
  // sum df_j^2 (1 + 2^-24)^n <= sum df_j^2 (1 + 2^-20).  Hence
  // d = ||x - q|| >= sqrt(sf / (1 + 2^-20)) /
  // (1 + 2^-24) - sqrt(n) e, and sf > (L + sqrt(n) e)^2 (1 + 2^-18) gives
  // d > L = sqrt(skip_d2 (1 + 2^-49)), so the double-precision d^2 (n + 1
  // roundings of 2^-53 each) exceeds skip_d2: such a pair is never counted.
  // The relative bounds need the float values in the normal range: the test
  // is used only for thresholds in [2^-100, 1e38] (below, the 2^-149
  // absolute rounding of subnormal squares is no longer negligible).
  float skip_f = INFINITY;
  if (max_abs >= 0 && max_abs < 1e30 && std::isfinite(skip_d2)) {
    const double e = 2.0 * max_abs * 0x1p-24 + 0x1p-148;
    const double L = std::sqrt(skip_d2 * (1.0 + 0x1p-49));
    const double lim_f = L + std::sqrt((double)n) * e;
    const double T = lim_f * lim_f * (1.0 + 0x1p-18);
    if (T < 1e38 && T >= 0x1p-100) {
      float tf = (float)T;
      if ((double)tf < T) tf = std::nextafter(tf, INFINITY);
      skip_f = tf;
    }
  }
  const int pts = pstride > 1 ? 1 : kPtsAll;
  int64_t want = ceil_div(ceil_div(N, pstride), (int64_t)kBlock * pts);
  int nb = (int)(want < 2048 ? want : 2048);
#define KNN_HIST(D, P) \
  k_dist_histogram<D, P><<<nb, kBlock, 0, s>>>(X, N, pstride, sample, ns, inv_bw, count_bins, \
                                               skip_d2, skip_f, counts)
  switch (n * 8 + pts) {
    case 2 * 8 + 1: KNN_HIST(2, 1); break;
    case 3 * 8 + 1: KNN_HIST(3, 1); break;
    case 4 * 8 + 1: KNN_HIST(4, 1); break;
    case 5 * 8 + 1: KNN_HIST(5, 1); break;
    case 6 * 8 + 1: KNN_HIST(6, 1); break;
    case 2 * 8 + kPtsAll: KNN_HIST(2, kPtsAll); break;
    case 3 * 8 + kPtsAll: KNN_HIST(3, kPtsAll); break;
    case 4 * 8 + kPtsAll: KNN_HIST(4, kPtsAll); break;
    case 5 * 8 + kPtsAll: KNN_HIST(5, kPtsAll); break;
    case 6 * 8 + kPtsAll: KNN_HIST(6, kPtsAll); break;
    default: throw Error(KNN_EINVAL, "dims out of range");
  }
#undef KNN_HIST
  KNN_LAUNCHED();
}

}  // namespace knn
