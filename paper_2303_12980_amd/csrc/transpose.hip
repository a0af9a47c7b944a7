// Pairs ordered by neighbour atom, for the adjoint of features at reference
// points: a point is no atom, so its pairs have no mirror entries, and each
// atom's gradient is gathered from the pairs that name it as neighbour.  A
// stable LSD radix sort of the pair indices by neighbour (8-bit digits, as
// many passes as the atom count needs) gives, for every atom, its pairs in
// ascending pair order; the gather then sums in that order, so the result
// does not depend on scheduling.  Stability inside a tile comes from
// wavefront match masks (ballots over the digit bits) and per-wavefront
// digit counts combined in wavefront order.
#include "gmp_internal.h"

namespace gmp {
namespace {

constexpr int kTileThreads = 256;
constexpr int kTileRounds = 16;
constexpr int kTile = kTileThreads * kTileRounds;  // items per tile
constexpr int kDigits = 256;

// keys[p] = neighbour of pair p for the written pairs, else the sentinel
// n_atoms (sorts last); vals[p] = p
__global__ void k_tr_init(NbrDev nb, int64_t n_centres, int64_t n_atoms, int64_t n, uint32_t *keys,
                          uint32_t *vals) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t total = nb.offsets[n_centres];
  const int64_t valid = total <= nb.capacity ? total : 0;  // overflowed lists: no pair is gathered
  uint32_t k = (uint32_t)n_atoms;
  if (p < valid) {
    const int32_t j = nb.j[p];
    k = (j >= 0 && (int64_t)j < n_atoms) ? (uint32_t)j : (uint32_t)n_atoms;
  }
  keys[p] = k;
  vals[p] = (uint32_t)p;
}

// per-tile digit histogram, digit-major: hist[d * n_tiles + tile]
__global__ __launch_bounds__(kTileThreads) void k_tr_hist(const uint32_t *keys, int64_t n, int shift,
                                                          int32_t *hist, int64_t n_tiles) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kTileRounds; ++r) {
    const int64_t p = t0 + r * kTileThreads + threadIdx.x;
    if (p < n) atomicAdd(&h[(keys[p] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// stable scatter of one tile: items in index order, round by round
__global__ __launch_bounds__(kTileThreads) void k_tr_scatter(const uint32_t *kin, const uint32_t *vin,
                                                             uint32_t *kout, uint32_t *vout, int64_t n, int shift,
                                                             const int64_t *off, int64_t n_tiles) {
  __shared__ int32_t run[kDigits];
  __shared__ int32_t wcnt[kTileThreads / kWave][kDigits];
  const int tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  run[tid] = 0;
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kTileRounds; ++r) {
    for (int k = 0; k < kTileThreads / kWave; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const int64_t p = t0 + r * kTileThreads + tid;
    const bool valid = p < n;
    uint32_t key = 0, val = 0;
    int d = 0;
    if (valid) {
      key = kin[p];
      val = vin[p];
      d = (int)((key >> shift) & 255u);
    }
    // lanes of this wavefront holding the same digit
    uint64_t mask = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot(((d >> b) & 1) != 0);
      mask &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int wrank = __popcll(mask & below);
    if (valid && wrank == 0) wcnt[w][d] = __popcll(mask);
    __syncthreads();
    if (valid) {
      int rank = run[d] + wrank;
      for (int k = 0; k < w; ++k) rank += wcnt[k][d];
      const int64_t dst = off[(int64_t)d * n_tiles + blockIdx.x] + rank;
      if (dst >= 0 && dst < n) {  // always, for counts that match the histogram pass
        kout[dst] = key;
        vout[dst] = val;
      }
    }
    __syncthreads();
    int add = 0;
    for (int k = 0; k < kTileThreads / kWave; ++k) add += wcnt[k][tid];
    run[tid] += add;
    __syncthreads();
  }
}

// start[a] = first sorted position whose key is >= a, for a in 0..n_atoms
__global__ void k_tr_starts(const uint32_t *keys, int64_t n, int64_t n_atoms, int64_t *start) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n) return;
  int64_t lo = t == 0 ? -1 : (int64_t)keys[t - 1];
  int64_t hi = t == n ? n_atoms : (int64_t)keys[t];
  lo = lo > n_atoms ? n_atoms : lo;  // keys never exceed n_atoms; kept inside start[] regardless
  hi = hi > n_atoms ? n_atoms : hi;
  for (int64_t a = lo + 1; a <= hi; ++a) start[a] = t;
}

}  // namespace

int64_t transpose_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

// Sorts the pair indices [0, n) by neighbour atom (stable).  Output: the
// pair order in vals_out and, for every atom a, the range
// [start[a], start[a+1]) of its pairs; pairs of unwritten lists sort last,
// past start[n_atoms].
void transpose_by_neighbour(const NbrDev &nb, int64_t n_centres, int64_t n_atoms, int64_t n, uint32_t *key_a,
                            uint32_t *key_b, uint32_t *val_a, uint32_t *val_b, int32_t *hist, int64_t *off,
                            int64_t *scan_aux, int64_t *start, uint32_t **vals_out, hipStream_t s) {
  int bits = 1;
  while (bits < 32 && ((uint64_t)n_atoms >> bits) != 0) ++bits;  // keys are <= n_atoms
  const int passes = (bits + 7) / 8;
  const int64_t tiles = transpose_tiles(n);
  uint32_t *kin = key_a, *kout = key_b, *vin = val_a, *vout = val_b;
  if (n > 0) {
    GMP_LAUNCH("adj_tr_init", k_tr_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nb, n_centres, n_atoms,
               n, kin, vin);
    for (int pass = 0; pass < passes; ++pass) {
      const int shift = 8 * pass;
      GMP_LAUNCH("adj_tr_hist", k_tr_hist, dim3((unsigned)tiles), dim3(kTileThreads), 0, s, kin, n, shift, hist,
                 tiles);
      scan_i32_to_i64(hist, off, kDigits * tiles, scan_aux, s);
      GMP_LAUNCH("adj_tr_scatter", k_tr_scatter, dim3((unsigned)tiles), dim3(kTileThreads), 0, s, kin, vin, kout,
                 vout, n, shift, off, tiles);
      uint32_t *t = kin; kin = kout; kout = t;
      t = vin; vin = vout; vout = t;
    }
  }
  GMP_LAUNCH("adj_tr_starts", k_tr_starts, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, kin, n, n_atoms,
             start);
  *vals_out = vin;
}

}  // namespace gmp
