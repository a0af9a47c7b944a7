// Small device utilities: zero fill and exclusive prefix sums.
//
// The scans are integer sums in a fixed order (one workgroup for short
// arrays, else a three-pass reduce / scan-of-block-sums / add scheme), so
// their results are deterministic, and no memset node is recorded when a
// caller captures the stream into a graph.
#include "gmp_internal.h"

namespace gmp {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ void k_fill_zero(uint32_t *p, size_t n_words) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n_words; i += stride) p[i] = 0u;
}

// block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *lds, int64_t *total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    int64_t add = t >= o ? lds[t - o] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int64_t incl = lds[t];
  *total = lds[kScanBlock - 1];
  __syncthreads();
  return incl - v;
}

template <typename Tin>
__global__ void k_scan_reduce(const Tin *in, int64_t n, int64_t *aux) {
  __shared__ int64_t lds[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  lds[threadIdx.x] = s;
  __syncthreads();
  for (int o = kScanBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) aux[blockIdx.x] = lds[0];
}

// single block: exclusive scan of the block sums in place, total at aux[nb]
__global__ void k_scan_aux(int64_t *aux, int64_t nb) {
  __shared__ int64_t lds[kScanBlock];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? aux[i] : 0;
    int64_t tot;
    int64_t ex = block_exclusive_scan(v, lds, &tot);
    if (i < nb) aux[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) aux[nb] = carry;
}

template <typename Tin>
__global__ void k_scan_apply(const Tin *in, int64_t *out, int64_t n, const int64_t *aux, int64_t nb) {
  __shared__ int64_t lds[kScanBlock];
  int64_t base = (int64_t)blockIdx.x * kScanTile;
  // thread t owns items base + t*kScanItems .. +kScanItems-1 (contiguous)
  int64_t vals[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    vals[k] = i < n ? (int64_t)in[i] : 0;
    s += vals[k];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(s, lds, &tot) + aux[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) out[i] = ex;
    ex += vals[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = aux[nb];
}

// Short arrays: one workgroup of 1024 threads walks tiles of 4096 items;
// each thread sums 4 contiguous items, wavefronts scan with shuffles, the
// 16 wavefront totals are scanned by the first wavefront, and a running
// carry joins the tiles.
constexpr int kSingleThreads = 1024;
constexpr int kSingleTile = kSingleThreads * 4;
constexpr int64_t kSingleMax = 65536;

template <typename Tin>
__global__ __launch_bounds__(kSingleThreads) void k_scan_single(const Tin *in, int64_t *out, int64_t n) {
  __shared__ int64_t wtot[kSingleThreads / kWave];
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += kSingleTile) {
    int64_t v[4];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + (int64_t)t * 4 + k;
      v[k] = i < n ? (int64_t)in[i] : 0;
      s += v[k];
    }
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wtot[w] = incl;
    __syncthreads();
    if (w == 0) {
      const int64_t x = lane < kSingleThreads / kWave ? wtot[lane] : 0;
      int64_t xi = x;
#pragma unroll
      for (int o = 1; o < kSingleThreads / kWave; o <<= 1) {
        const int64_t y = __shfl_up(xi, o, kWave);
        if (lane >= o) xi += y;
      }
      if (lane < kSingleThreads / kWave) wtot[lane] = xi - x;  // exclusive wavefront offsets
    }
    __syncthreads();
    int64_t ex = carry + wtot[w] + (incl - s);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = base + (int64_t)t * 4 + k;
      if (i < n) out[i] = ex;
      ex += v[k];
    }
    // the tile total: last thread's inclusive end
    if (t == kSingleThreads - 1) wtot[0] = ex - carry;
    __syncthreads();
    carry += wtot[0];
    __syncthreads();
  }
  if (t == 0) out[n] = carry;
}

template <typename Tin>
void scan_impl(const Tin *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s) {
  if (n <= kSingleMax) {
    auto one = k_scan_single<Tin>;
    GMP_LAUNCH("scan_single", one, dim3(1), dim3(kSingleThreads), 0, s, in, out, n);
    return;
  }
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) nb = 1;
  auto red = k_scan_reduce<Tin>;
  auto app = k_scan_apply<Tin>;
  GMP_LAUNCH("scan_reduce", red, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, aux);
  GMP_LAUNCH("scan_aux", k_scan_aux, dim3(1), dim3(kScanBlock), 0, s, aux, nb);
  GMP_LAUNCH("scan_apply", app, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n, aux, nb);
}

}  // namespace

int64_t scan_aux_size(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

void scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, aux, s);
}

void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s) {
  scan_impl<int64_t>(in, out, n, aux, s);
}

__global__ void k_fill_zero3(uint32_t *p0, size_t n0, uint32_t *p1, size_t n1, uint32_t *p2, size_t n2) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n0 + n1 + n2; i += stride) {
    if (i < n0) p0[i] = 0u;
    else if (i < n0 + n1) p1[i - n0] = 0u;
    else p2[i - n0 - n1] = 0u;
  }
}

void fill_zero3(void *p0, size_t b0, void *p1, size_t b1, void *p2, size_t b2, hipStream_t s) {
  const size_t w0 = (b0 + 3) / 4, w1 = (b1 + 3) / 4, w2 = (b2 + 3) / 4;
  const size_t words = w0 + w1 + w2;
  if (words == 0) return;
  size_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  GMP_LAUNCH("fill_zero", k_fill_zero3, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p0, w0, (uint32_t *)p1,
             w1, (uint32_t *)p2, w2);
}

void fill_zero(void *p, size_t bytes, hipStream_t s) {
  size_t words = (bytes + 3) / 4;
  if (words == 0) return;
  size_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  GMP_LAUNCH("fill_zero", k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, words);
}

}  // namespace gmp
