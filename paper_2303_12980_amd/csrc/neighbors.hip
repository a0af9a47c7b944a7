// Neighbour build: lattice wrap, cell-list binning, per-centre count, fill
// and canonical sort, reverse-pair index.
//
// The cutoff is inferred from the overlap threshold (the paper's "Examples"
// section): a pair (j, n) belongs to centre i when its squared distance q is
// at most the largest rc(sigma)^2.  Image shifts n range over every lattice
// translation on periodic axes, so atoms (and the centre itself) appear as
// often as they fit inside the cutoff sphere.
//
// Floating point: reciprocal rows, fractional coordinates, wrap, image
// shifts, displacements and q are FP64 in a fixed operation order with no
// contraction (the file is built with -ffp-contract=off), so every kernel that
// recomputes q gets the same bits and (j,i,-n) has exactly the q of (i,j,n).
//
// Cell list: fractional space of each structure is cut into nb_k bins per
// periodic axis (edge ~ rc_max / bin_divisor); a centre visits the "virtual"
// bins V_k in [floor((f_k - reach_k) nb_k), floor((f_k + reach_k) nb_k)],
// each of which is real bin V mod nb with image shift floor(V / nb).  Atoms
// are stored bin-sorted in SoA arrays so a bin is read with coalesced loads.
#include "gmp_internal.h"

namespace gmp {
namespace {

__device__ inline void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

__device__ inline int floordiv(int a, int b) { int q = a / b; return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q; }
__device__ inline int pmod(int a, int b) { int r = a % b; return r < 0 ? r + b : r; }

__global__ void k_struct_setup(BatchDev bt, StructInfo *info, double rcmax, int bin_div, uint32_t *status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= bt.n_structs) return;
  StructInfo I;
  const int pbc = bt.pbc[s] & 7;
  const int64_t n_s = bt.atom_offsets[s + 1] - bt.atom_offsets[s];
  I.pbc = pbc;
  I.bin_base = bt.atom_offsets[s] + s;
  for (int k = 0; k < 9; ++k) I.b[k] = 0.0;
  for (int k = 0; k < 3; ++k) { I.nb[k] = 1; I.reach[k] = 0.0; }
  if (pbc) {
    const double *a = bt.cell + 9 * (int64_t)s;
    double c23[3], c31[3], c12[3];
    cross3(a + 3, a + 6, c23);
    cross3(a + 6, a, c31);
    cross3(a, a + 3, c12);
    double V = dot3(a, c23);
    bool ok = isfinite(V) && V != 0.0;
    for (int k = 0; k < 9; ++k) ok = ok && isfinite(a[k]);
    if (!ok) {
      atomicOr(status, ST_CELL);
    } else {
      for (int k = 0; k < 3; ++k) { I.b[k] = c23[k] / V; I.b[3 + k] = c31[k] / V; I.b[6 + k] = c12[k] / V; }
      const double ell = rcmax / (double)bin_div;
      for (int k = 0; k < 3; ++k) {
        if (!(pbc & (1 << k))) continue;
        double inv_h = sqrt(dot3(I.b + 3 * k, I.b + 3 * k));
        double h = 1.0 / inv_h;
        double nbk = ell > 0.0 ? floor(h / ell) : 1.0;
        if (!(nbk >= 1.0)) nbk = 1.0;
        if (nbk > 1024.0) nbk = 1024.0;
        I.nb[k] = (int)nbk;
        I.reach[k] = rcmax * inv_h * (1.0 + 1e-12) + 1e-12;
        // image shifts must fit a signed byte
        if (I.reach[k] + 2.0 > 126.0) atomicOr(status, ST_SHIFT_RANGE);
      }
      // never more bins than atoms (bin slots per structure are n_s + 1)
      int64_t cap = n_s > 1 ? n_s : 1;
      while ((int64_t)I.nb[0] * I.nb[1] * I.nb[2] > cap) {
        int kk = 0;
        if (I.nb[1] > I.nb[kk]) kk = 1;
        if (I.nb[2] > I.nb[kk]) kk = 2;
        I.nb[kk] = I.nb[kk] > 1 ? (I.nb[kk] + 1) / 2 : 1;
      }
    }
  }
  info[s] = I;
}

__global__ void k_wrap(BatchDev bt, const StructInfo *info, NbrDev nb, double *fw, int32_t *bin_of,
                       int32_t *bin_count, int n_elements, uint32_t *status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.n_atoms) return;
  {
    const int sp = bt.species[i];
    if (sp < 0 || sp >= n_elements) atomicOr(status, ST_SPECIES);
  }
  const int64_t N = bt.n_atoms;
  const int s = struct_of_atom(bt.atom_offsets, bt.n_structs, i);
  const StructInfo &I = info[s];
  const double R[3] = {bt.x[i], bt.y[i], bt.z[i]};
  if (!(isfinite(R[0]) && isfinite(R[1]) && isfinite(R[2]))) atomicOr(status, ST_NONFINITE);
  int m[3] = {0, 0, 0};
  int b[3] = {0, 0, 0};
  double f3[3] = {0.0, 0.0, 0.0};
  double rwv[3] = {R[0], R[1], R[2]};
  if (I.pbc) {
    const double *a = bt.cell + 9 * (int64_t)s;
    for (int k = 0; k < 3; ++k) {
      if (!(I.pbc & (1 << k))) continue;
      double f = dot3(R, I.b + 3 * k);
      if (!(fabs(f) < 1.0e9)) { atomicOr(status, ST_NONFINITE); f = 0.0; }
      double fl = floor(f);
      m[k] = (int)fl;
      double w = f - fl;  // exact, in [0, 1)
      f3[k] = w;
      int bk = (int)(w * (double)I.nb[k]);
      if (bk > I.nb[k] - 1) bk = I.nb[k] - 1;
      if (bk < 0) bk = 0;
      b[k] = bk;
    }
    for (int c = 0; c < 3; ++c) {
      double t = (double)m[0] * a[c] + (double)m[1] * a[3 + c];
      t = t + (double)m[2] * a[6 + c];
      rwv[c] = R[c] - t;
    }
  }
  nb.rw[i] = rwv[0];
  nb.rw[N + i] = rwv[1];
  nb.rw[2 * N + i] = rwv[2];
  nb.wrap[3 * i] = m[0];
  nb.wrap[3 * i + 1] = m[1];
  nb.wrap[3 * i + 2] = m[2];
  fw[i] = f3[0];
  fw[N + i] = f3[1];
  fw[2 * N + i] = f3[2];
  int64_t bin = I.bin_base + ((int64_t)b[0] * I.nb[1] + b[1]) * I.nb[2] + b[2];
  bin_of[i] = (int32_t)bin;
  atomicAdd(&bin_count[bin], 1);
}

__global__ void k_scatter(BatchDev bt, NbrDev nb, const int32_t *bin_of, const int64_t *bin_start,
                          int32_t *bin_fill, double *sx, double *sy, double *sz, int32_t *sid,
                          int32_t *ssp, int n_elements) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bt.n_atoms) return;
  const int64_t N = bt.n_atoms;
  int32_t b = bin_of[i];
  int64_t p = bin_start[b] + atomicAdd(&bin_fill[b], 1);
  sx[p] = nb.rw[i];
  sy[p] = nb.rw[N + i];
  sz[p] = nb.rw[2 * N + i];
  sid[p] = (int32_t)i;
  int sp = bt.species[i];
  ssp[p] = sp < 0 ? 0 : (sp >= n_elements ? n_elements - 1 : sp);  // out-of-range species are flagged in k_wrap
}

// Range of virtual bins along axis k for a centre at fractional f.
__device__ inline void vrange(const StructInfo &I, int k, double f, int &lo, int &hi) {
  if (!(I.pbc & (1 << k))) { lo = hi = 0; return; }
  double nbk = (double)I.nb[k];
  lo = (int)floor((f - I.reach[k]) * nbk - 1e-6);
  hi = (int)floor((f + I.reach[k]) * nbk + 1e-6);
}

struct Cand {
  const StructInfo *I;
  const double *cell;
  int lo[3], hi[3], nv[3];
  int total;
};

__device__ inline void cand_setup(Cand &C, const StructInfo *info, const BatchDev &bt, int s,
                                  const double *fw, int64_t i) {
  const int64_t N = bt.n_atoms;
  C.I = info + s;
  C.cell = bt.cell + 9 * (int64_t)s;
  const double f[3] = {fw[i], fw[N + i], fw[2 * N + i]};
  C.total = 1;
  for (int k = 0; k < 3; ++k) {
    vrange(*C.I, k, f[k], C.lo[k], C.hi[k]);
    C.nv[k] = C.hi[k] - C.lo[k] + 1;
    C.total *= C.nv[k];
  }
}

// virtual bin v (linear index) -> real bin slot and image shift
__device__ inline int64_t cand_bin(const Cand &C, int v, int n[3]) {
  int r[3];
  int t = v;
  r[2] = t % C.nv[2]; t /= C.nv[2];
  r[1] = t % C.nv[1]; t /= C.nv[1];
  r[0] = t;
  int b[3];
  for (int k = 0; k < 3; ++k) {
    int V = C.lo[k] + r[k];
    int nbk = C.I->nb[k];
    b[k] = pmod(V, nbk);
    n[k] = floordiv(V, nbk);
  }
  return C.I->bin_base + ((int64_t)b[0] * C.I->nb[1] + b[1]) * C.I->nb[2] + b[2];
}

__device__ inline int shell_of(const PlanDev &P, double q) {
  int sh = 0;
  for (int s = 0; s < P.S; ++s) sh += (P.rc2[s] < q) ? 1 : 0;
  return sh;
}

// One wavefront per centre: count neighbours per (species, shell) bucket.
__global__ __launch_bounds__(256) void k_count(PlanDev P, BatchDev bt, NbrDev nb, const StructInfo *info,
                                               const double *fw, const int64_t *bin_start,
                                               const double *sx, const double *sy, const double *sz,
                                               const int32_t *ssp, int32_t *cnt, int64_t *ptotal,
                                               uint32_t *status) {
  extern __shared__ int32_t lds_cnt[];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int nbk = P.E * P.S;
  int32_t *c = lds_cnt + w * nbk;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + w;
  const int64_t N = bt.n_atoms;
  for (int t = lane; t < nbk; t += kWave) c[t] = 0;
  wave_lds_sync();
  if (i < N) {
    const int s = struct_of_atom(bt.atom_offsets, bt.n_structs, i);
    Cand C;
    cand_setup(C, info, bt, s, fw, i);
    const double rix = nb.rw[i], riy = nb.rw[N + i], riz = nb.rw[2 * N + i];
    for (int v = 0; v < C.total; ++v) {
      int n[3];
      int64_t bin = cand_bin(C, v, n);
      double shx = 0.0, shy = 0.0, shz = 0.0;
      if (C.I->pbc) image_shift(C.cell, n[0], n[1], n[2], shx, shy, shz);
      const int64_t b0 = bin_start[bin], b1 = bin_start[bin + 1];
      for (int64_t t = b0 + lane; t < b1; t += kWave) {
        double dx = (sx[t] - rix) + shx;
        double dy = (sy[t] - riy) + shy;
        double dz = (sz[t] - riz) + shz;
        double q = (dx * dx + dy * dy) + dz * dz;
        if (q <= P.rcmax2) atomicAdd(&c[shell_of(P, q) * P.E + ssp[t]], 1);
      }
    }
  }
  wave_lds_sync();
  if (i < N) {
    int64_t tot = 0;
    for (int t = lane; t < nbk; t += kWave) {
      cnt[i * nbk + t] = c[t];
      tot += c[t];
    }
    for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o, kWave);
    if (lane == 0) {
      ptotal[i] = tot;
      atomicMax(status + 4, (uint32_t)(tot > 0x7fffffff ? 0x7fffffff : tot));
    }
  }
}

__device__ inline void cmpswap(uint64_t *a, int i, int l) {
  uint64_t x = a[i], y = a[l];
  if (x > y) { a[i] = y; a[l] = x; }
}

// Sort a[0..n) ascending by one wavefront: bitonic network whose first
// merge stage compares mirror pairs, so every comparator is ascending and
// indices >= n act as +infinity without being touched.
__device__ void wave_sort(uint64_t *a, int n) {
  const int lane = lane_id();
  if (n <= 1) return;
  if (n <= kWave) {
    uint64_t k = lane < n ? a[lane] : ~0ull;
    for (int size = 2; size <= kWave; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        uint64_t o = __shfl_xor(k, stride, kWave);
        bool up = (lane & size) == 0;
        bool lower = (lane & stride) == 0;
        uint64_t mn = k < o ? k : o, mx = k < o ? o : k;
        k = (lower == up) ? mn : mx;
      }
    if (lane < n) a[lane] = k;
    wave_lds_sync();
    return;
  }
  int p2 = 1;
  while (p2 < n) p2 <<= 1;
  const int half = p2 >> 1;
  for (int k = 2; k <= p2; k <<= 1) {
    const int hk = k >> 1;
    for (int t = lane; t < half; t += kWave) {
      int blk = t / hk, off = t - blk * hk;
      int i = blk * k + off, l = blk * k + k - 1 - off;
      if (l < n) cmpswap(a, i, l);
    }
    wave_lds_sync();
    for (int j = k >> 2; j >= 1; j >>= 1) {
      for (int t = lane; t < half; t += kWave) {
        int blk = t / j, off = t - blk * j;
        int i = blk * 2 * j + off, l = i + j;
        if (l < n) cmpswap(a, i, l);
      }
      wave_lds_sync();
    }
  }
}

__device__ inline uint64_t make_key(int64_t j, int n1, int n2, int n3) {
  return ((uint64_t)j << 24) | ((uint64_t)(n1 + 128) << 16) | ((uint64_t)(n2 + 128) << 8) | (uint64_t)(n3 + 128);
}

// One workgroup per centre: fill its buckets (shell h, species e), in
// bucket order h * E + e, in LDS; sort every bucket by (j, n); write j /
// shift, the bucket starts and the sigma-prefix ends.
__global__ __launch_bounds__(256) void k_fill(PlanDev P, BatchDev bt, NbrDev nb, const StructInfo *info,
                                              const double *fw, const int64_t *bin_start,
                                              const double *sx, const double *sy, const double *sz,
                                              const int32_t *sid, const int32_t *ssp, const int32_t *cnt,
                                              int lds_keys, uint32_t *status) {
  extern __shared__ uint64_t lds_u64[];
  const int nbk = P.E * P.S;
  uint64_t *keys = lds_u64;
  int32_t *bstart = (int32_t *)(lds_u64 + lds_keys);  // [nbk+1]
  int32_t *cursor = bstart + nbk + 1;                 // [nbk]
  const int64_t i = blockIdx.x;
  const int64_t N = bt.n_atoms;
  const int tid = threadIdx.x, w = tid / kWave, nw = blockDim.x / kWave, lane = lane_id();
  const int64_t base = nb.offsets[i];
  const int64_t total = nb.offsets[i + 1] - base;
  const bool overflow = nb.offsets[i + 1] > nb.capacity;
  const bool too_big = total > lds_keys;
  if (tid == 0) {
    int32_t acc = 0;
    for (int b = 0; b < nbk; ++b) { bstart[b] = acc; acc += cnt[i * nbk + b]; }
    bstart[nbk] = acc;
    if (overflow) atomicOr(status, ST_OVERFLOW);
    if (too_big) atomicOr(status, ST_SORT_SIZE);
    if ((int64_t)acc != total) atomicOr(status, ST_INTERNAL);
  }
  __syncthreads();
  for (int b = tid; b <= nbk; b += blockDim.x) nb.bucket_start[i * (nbk + 1) + b] = bstart[b];
  for (int s = tid; s < P.S; s += blockDim.x) nb.sigma_end[i * P.S + s] = bstart[(P.rank_lt[s] + 1) * P.E];
  if (overflow || too_big) return;
  for (int b = tid; b < nbk; b += blockDim.x) cursor[b] = bstart[b];
  __syncthreads();
  const int s = struct_of_atom(bt.atom_offsets, bt.n_structs, i);
  Cand C;
  cand_setup(C, info, bt, s, fw, i);
  const double rix = nb.rw[i], riy = nb.rw[N + i], riz = nb.rw[2 * N + i];
  for (int v = w; v < C.total; v += nw) {
    int n[3];
    int64_t bin = cand_bin(C, v, n);
    double shx = 0.0, shy = 0.0, shz = 0.0;
    if (C.I->pbc) image_shift(C.cell, n[0], n[1], n[2], shx, shy, shz);
    const int64_t b0 = bin_start[bin], b1 = bin_start[bin + 1];
    for (int64_t t = b0 + lane; t < b1; t += kWave) {
      double dx = (sx[t] - rix) + shx;
      double dy = (sy[t] - riy) + shy;
      double dz = (sz[t] - riz) + shz;
      double q = (dx * dx + dy * dy) + dz * dz;
      if (q <= P.rcmax2) {
        int bk = shell_of(P, q) * P.E + ssp[t];
        int pos = atomicAdd(&cursor[bk], 1);
        if (pos < bstart[bk + 1]) keys[pos] = make_key(sid[t], n[0], n[1], n[2]);
        else atomicOr(status, ST_INTERNAL);
      }
    }
  }
  __syncthreads();
  for (int b = w; b < nbk; b += nw) {
    const int b0 = bstart[b], bn = bstart[b + 1] - b0;
    if (bn == 0) continue;
    wave_sort(keys + b0, bn);
    const int e = b % P.E;
    for (int t = lane; t < bn; t += kWave) {
      uint64_t k = keys[b0 + t];
      int32_t jj = (int32_t)(k >> 24);
      uint32_t n1 = (uint32_t)(((k >> 16) & 0xff) - 128) & 0xffu;
      uint32_t n2 = (uint32_t)(((k >> 8) & 0xff) - 128) & 0xffu;
      uint32_t n3 = (uint32_t)((k & 0xff) - 128) & 0xffu;
      nb.j[base + b0 + t] = jj;
      nb.shift[base + b0 + t] = (int32_t)(n1 | (n2 << 8) | (n3 << 16) | ((uint32_t)e << 24));
    }
  }
}

// Reverse index: for pair (i, j, n) find (j, i, -n) in j's list by binary
// search inside j's bucket (shell of q, species of i).
__global__ __launch_bounds__(256) void k_reverse(PlanDev P, BatchDev bt, NbrDev nb, uint32_t *status) {
  const int64_t N = bt.n_atoms;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= N) return;
  const int lane = lane_id();
  const int nbk = P.E * P.S;
  const int s = struct_of_atom(bt.atom_offsets, bt.n_structs, i);
  const double *cell = bt.cell + 9 * (int64_t)s;
  const int pbc = bt.pbc[s] & 7;
  const int64_t base = nb.offsets[i], end = nb.offsets[i + 1];
  if (end > nb.capacity) return;
  int ei = bt.species[i];
  ei = ei < 0 ? 0 : (ei >= P.E ? P.E - 1 : ei);
  const double rix = nb.rw[i], riy = nb.rw[N + i], riz = nb.rw[2 * N + i];
  for (int64_t p = base + lane; p < end; p += kWave) {
    const int32_t j = nb.j[p];
    const int32_t w = nb.shift[p];
    const int n1 = shift_n(w, 0), n2 = shift_n(w, 1), n3 = shift_n(w, 2);
    double shx = 0.0, shy = 0.0, shz = 0.0;
    if (pbc) image_shift(cell, n1, n2, n3, shx, shy, shz);
    double dx = (nb.rw[j] - rix) + shx;
    double dy = (nb.rw[N + j] - riy) + shy;
    double dz = (nb.rw[2 * N + j] - riz) + shz;
    double q = (dx * dx + dy * dy) + dz * dz;
    const int b = shell_of(P, q) * P.E + ei;
    const int32_t *bs = nb.bucket_start + (int64_t)j * (nbk + 1);
    int lo = bs[b], hi = bs[b + 1];
    const uint64_t key = make_key(i, -n1, -n2, -n3);
    const int64_t jb = nb.offsets[j];
    int found = -1;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      const int32_t wm = nb.shift[jb + mid];
      uint64_t km = make_key(nb.j[jb + mid], shift_n(wm, 0), shift_n(wm, 1), shift_n(wm, 2));
      if (km == key) { found = mid; break; }
      if (km < key) lo = mid + 1; else hi = mid;
    }
    if (found < 0) atomicOr(status, ST_INTERNAL);
    nb.reverse[p] = found;
  }
}

}  // namespace

// ------------------------------------------------------------------ host launchers
void launch_struct_setup(const gmp_plan *p, const BatchDev &bt, const WsLayout &L, hipStream_t s) {
  int nb = (bt.n_structs + 63) / 64;
  double rcmax = sqrt(p->dev.rcmax2);
  GMP_LAUNCH("nbr_struct_setup", k_struct_setup, dim3(nb), dim3(64), 0, s, bt, L.sinfo, rcmax,
             p->tuning.bin_divisor, L.status);
}

void launch_wrap(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s) {
  int64_t blocks = (bt.n_atoms + 255) / 256;
  GMP_LAUNCH("nbr_wrap", k_wrap, dim3((unsigned)blocks), dim3(256), 0, s, bt, L.sinfo, nb, L.fw, L.bin_of,
             L.bin_count, n_elements, L.status);
}

void launch_scatter(const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int n_elements, hipStream_t s) {
  int64_t blocks = (bt.n_atoms + 255) / 256;
  GMP_LAUNCH("nbr_scatter", k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, bt, nb, L.bin_of,
             L.bin_start, L.bin_fill, L.sx, L.sy, L.sz, L.sid, L.ssp, n_elements);
}

void launch_count(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, hipStream_t s) {
  int64_t blocks = (bt.n_atoms + 3) / 4;
  size_t smem = sizeof(int32_t) * 4 * p->dev.E * p->dev.S;
  GMP_LAUNCH("nbr_count", k_count, dim3((unsigned)blocks), dim3(256), smem, s, p->dev, bt, nb, L.sinfo, L.fw,
             L.bin_start, L.sx, L.sy, L.sz, L.ssp, L.cnt, L.ptotal, L.status);
}

void launch_fill(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, int lds_keys,
                 hipStream_t s) {
  int nbk = p->dev.E * p->dev.S;
  size_t smem = sizeof(uint64_t) * lds_keys + sizeof(int32_t) * (2 * nbk + 2);
  GMP_LAUNCH("nbr_fill_sort", k_fill, dim3((unsigned)bt.n_atoms), dim3(256), smem, s, p->dev, bt, nb, L.sinfo,
             L.fw, L.bin_start, L.sx, L.sy, L.sz, L.sid, L.ssp, L.cnt, lds_keys, L.status);
}

void launch_reverse(const gmp_plan *p, const BatchDev &bt, const NbrDev &nb, const WsLayout &L, hipStream_t s) {
  int64_t blocks = (bt.n_atoms + 3) / 4;
  GMP_LAUNCH("nbr_reverse", k_reverse, dim3((unsigned)blocks), dim3(256), 0, s, p->dev, bt, nb, L.status);
}

}  // namespace gmp
