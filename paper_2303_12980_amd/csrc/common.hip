// Small device utilities: zero fill and exclusive prefix sums.
//
// The scans are a three-pass reduce / scan-of-block-sums / add scheme with
// a fixed summation order, so their results are deterministic and no
// memset node is recorded when a caller captures the stream into a graph.
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

template <typename Tin>
void scan_impl(const Tin *in, int64_t *out, int64_t n, int64_t *aux, hipStream_t s) {
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

void fill_zero(void *p, size_t bytes, hipStream_t s) {
  size_t words = (bytes + 3) / 4;
  if (words == 0) return;
  size_t blocks = (words + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  GMP_LAUNCH("fill_zero", k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p, words);
}

}  // namespace gmp
