// Cell binning, deterministic cell sort, per-site records and real-space
// neighbour lists.
//
// Sites are binned into cells of edge >= cutoff/2 (a 5x5x5 cell stencil
// then covers the cutoff sphere), counting-sorted by cell, and each cell's
// segment is sorted by caller index so that the order -- and with it every
// summation order downstream -- is reproducible.  The neighbour-list kernel
// runs one wavefront per cell: 64 candidate sites are loaded per step and
// tested against every site of the cell; hits are compacted with ballots so
// list order is deterministic too.  Four ELL lists are produced:
//   all   intermolecular site pairs within the cutoff (E, E_elec, forces)
//   in    same-molecule site pairs (excluded or damped, always present)
//   pol   intermolecular polarizable pairs within the cutoff (T)
//   ipol  same-molecule polarizable pairs (T, Thole-damped)
#include <algorithm>
#include <initializer_list>
#include <utility>

#include "common.h"
#include "nlist.h"

namespace sibfa {

// ------------------------------------------------------------ fill / scan
template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

static int fill_blocks(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_fill_int(int* p, int v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill<int>, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, v, n);
}
void launch_fill_double(double* p, double v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill<double>, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, v, n);
}
void launch_fill_float(float* p, float v, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill<float>, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, v, n);
}

// Several int buffers set to one value in a single launch.
__global__ void k_fill_ints(FillList f) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int k = 0; k < f.n; ++k)
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.cnt[k]; i += stride)
      f.p[k][i] = f.v;
}

void launch_fill_ints(std::initializer_list<std::pair<int*, size_t>> bufs, int v, hipStream_t s) {
  FillList f{};
  size_t mx = 0;
  for (const auto& b : bufs) {
    if (f.n == kFillMax) {   // more than one launch's worth
      hipLaunchKernelGGL(k_fill_ints, dim3(fill_blocks(mx)), dim3(kBlock), 0, s, f);
      f.n = 0;
      mx = 0;
    }
    f.p[f.n] = b.first;
    f.cnt[f.n] = b.second;
    ++f.n;
    mx = std::max(mx, b.second);
  }
  f.v = v;
  if (f.n && mx) hipLaunchKernelGGL(k_fill_ints, dim3(fill_blocks(mx)), dim3(kBlock), 0, s, f);
}

constexpr int kScanTile = 4 * kBlock;   // elements per block

__device__ int block_exclusive_scan(int v, int* total) {
  __shared__ int wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ void k_scan_tiles(const int* in, int* out, int n, int* tile_sums) {
  const int base = blockIdx.x * kScanTile + threadIdx.x * 4;
  int v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int ex = block_exclusive_scan(s, &total);
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int* out, int n, const int* tile_offsets) {
  const int base = blockIdx.x * kScanTile + threadIdx.x * 4;
  const int add = tile_offsets[blockIdx.x];
  for (int k = 0; k < 4; ++k)
    if (base + k < n) out[base + k] += add;
}

// Exclusive scan of up to kScanSingleMax (16,384) values by one 1,024-thread
// workgroup: tiles of 4,096 values in order, each scanned in registers and
// across the wavefronts, with the running total carried to the next tile.
// One launch instead of the three of the multi-block form.
constexpr int kScanBig = 1024;
constexpr int kScanSingleMax = 4 * 4 * kScanBig;   // larger scans: the multi-block form is faster
__global__ __launch_bounds__(kScanBig) void k_scan_single(const int* in, int* out, int n) {
  __shared__ int wsum[kScanBig / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int carry = 0;
  for (int t0 = 0; t0 < n; t0 += 4 * kScanBig) {
    const int base = t0 + threadIdx.x * 4;
    int v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = (base + k < n) ? in[base + k] : 0;
      sum += v[k];
    }
    int x = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int wbase = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBig / 64; ++w) {
      if (w < wid) wbase += wsum[w];
      tot += wsum[w];
    }
    __syncthreads();   // wsum is rewritten by the next tile
    int ex = carry + wbase + x - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (base + k < n) out[base + k] = ex;
      ex += v[k];
    }
    carry += tot;
  }
}

size_t scan_temp_ints(int n) {
  const size_t tiles = (size_t)(n + kScanTile - 1) / kScanTile;
  if (tiles <= 1) return 1;
  return 2 * tiles + scan_temp_ints((int)tiles);
}

void launch_exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t s) {
  if (n <= 0) return;
  const int tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles > 1 && n <= kScanSingleMax) {
    hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kScanBig), 0, s, in, out, n);
    return;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, in, out, n, tmp);
  if (tiles == 1) return;
  launch_exclusive_scan(tmp, tmp + tiles, tiles, tmp + 2 * tiles, s);
  hipLaunchKernelGGL(k_scan_add, dim3(tiles), dim3(kBlock), 0, s, out, n,
                     (const int*)(tmp + tiles));
}

// ------------------------------------------------------------ binning
// Coordinate wrapped into [0, L).  Coordinates beyond kMaxBoxes box edges
// (rejected by the binning: the wrap has lost its precision there) map to
// 0, so that work queued before the error is read back indexes in bounds.
constexpr double kMaxBoxes = 1e6;
__device__ __forceinline__ double wrap(double x, double L, double iL) {
  double w = x - L * floor(x * iL);
  w = (w >= L) ? w - L : w;
  return (w > -L && w < L) ? w : 0.0;
}

// Neighbouring caller indices are usually neighbouring sites (a molecule's
// sites, molecules laid out in space order), so the counters are
// incremented per wavefront run of equal keys.
__global__ void k_bin(BinArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = c < a.n;
  int cell = 0, m = -1;
  if (act) {
    const double x0 = a.xyz[3 * c], x1 = a.xyz[3 * c + 1], x2 = a.xyz[3 * c + 2];
    if (!isfinite(x0) || !isfinite(x1) || !isfinite(x2)) atomicOr(a.err, 8);
    if (a.periodic && !(fabs(x0) <= kMaxBoxes * a.box[0] && fabs(x1) <= kMaxBoxes * a.box[1] &&
                        fabs(x2) <= kMaxBoxes * a.box[2]))
      atomicOr(a.err, 8);
    if (a.periodic) {
      int ci[3];
      for (int d = 0; d < 3; ++d) {
        double w = wrap(a.xyz[3 * c + d], a.box[d], a.ibox[d]);
        int k = (int)(w * a.nc[d] * a.ibox[d]);
        ci[d] = k >= a.nc[d] ? a.nc[d] - 1 : (k < 0 ? 0 : k);
      }
      cell = ci[0] + a.nc[0] * (ci[1] + a.nc[1] * ci[2]);
    }
    a.cell_of[c] = cell;
    m = a.mol[c];
    if (!(m >= 0 && m < a.n)) atomicOr(a.err, 2);
  }
  wave_atomic_inc(a.cell_count, cell, act);
  wave_atomic_inc(a.mol_count, m, act && m >= 0 && m < a.n);
}

// Slots within a key come from wavefront runs and one atomic per run; their
// order across wavefronts is fixed afterwards by k_sort_cells.
__global__ void k_scatter(const int* cell_of, const int* cell_start, int* cursor,
                          int* perm, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = c < n;
  const int cell = act ? cell_of[c] : 0;
  const int slot = wave_atomic_inc(cursor, cell, act);
  if (act) perm[cell_start[cell] + slot] = c;
}

// One thread per cell: insertion sort of the cell's segment by caller index.
// Sorts each cell's entries of perm (distinct site indices) in increasing
// order, which makes the cell-sorted order independent of the order in
// which the scatter's atomics ran.  One wavefront per cell: the entries are
// ranked in LDS (rank = number of smaller entries); cells too large for the
// LDS buffer fall back to an insertion sort by one lane.
constexpr int kSortLds = 256;
__global__ __launch_bounds__(64) void k_sort_cells(const int* cell_start, int ncell, int* perm) {
  __shared__ int v[kSortLds];
  const int cell = blockIdx.x;
  if (cell >= ncell) return;
  const int s = cell_start[cell], e = cell_start[cell + 1], n = e - s;
  if (n <= kSortLds) {
    for (int k = threadIdx.x; k < n; k += 64) v[k] = perm[s + k];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 64) {
      const int x = v[k];
      int r = 0;
      for (int m = 0; m < n; ++m) r += v[m] < x ? 1 : 0;
      perm[s + r] = x;
    }
  } else if (threadIdx.x == 0) {
    for (int i = s + 1; i < e; ++i) {
      const int x = perm[i];
      int j = i - 1;
      while (j >= s && perm[j] > x) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = x;
    }
  }
}

__global__ void k_sum_ints(const int* v, int n, unsigned long long* out) {
  unsigned long long m = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    m += (unsigned long long)v[i];
  for (int off = 32; off > 0; off >>= 1) m += __shfl_xor(m, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, m);
}

void launch_sum_ints(const int* v, int n, unsigned long long* out, hipStream_t s) {
  int blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_sum_ints, dim3(blocks), dim3(kBlock), 0, s, v, n, out);
}

void launch_bin(const BinArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_bin, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}
void launch_scatter(const int* cell_of, const int* cell_start, int* cursor, int* perm,
                    int n, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     cell_of, cell_start, cursor, perm, n);
}
void launch_sort_cells(const int* cell_start, int ncell, int* perm, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_cells, dim3(ncell), dim3(64), 0, s, cell_start, ncell, perm);
}
// ------------------------------------------------------------ records
// Positions (wrapped when periodic) and molecule ids in sorted order; the
// inverse permutation.  A non-finite coordinate (flagged by the binning, the
// call then fails) is stored as 0 and an out-of-range molecule id as 0, so
// that every kernel queued before the error is read back indexes in bounds.
__device__ __forceinline__ void rec_pos_of(const RecArgs& a, int i, int c, double xyz[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v = a.xyz[3 * c + k];
    if (!isfinite(v)) v = 0.0;
    if (a.periodic) v = wrap(v, a.box[k], a.ibox[k]);
    xyz[k] = v;
  }
  const int m = a.mol[c];
  a.mol_s[i] = (m >= 0 && m < a.n) ? m : 0;
  a.inv_perm[c] = i;
}
// Multipoles of caller site c: q, d, Theta (zero where not given).
__device__ __forceinline__ void rec_mult_of(const RecArgs& a, int c, double& q, double d[3],
                                            double t[6]) {
  q = a.q ? a.q[c] : 0.0;
  for (int k = 0; k < 3; ++k) d[k] = a.dip ? a.dip[3 * c + k] : 0.0;
  for (int k = 0; k < 6; ++k) t[k] = a.quad ? a.quad[6 * c + k] : 0.0;
}
__device__ __forceinline__ void rec_mult_store(const RecArgs& a, int i, const double d[3],
                                               const double t[6]) {
  a.sth[i] = make_double4(t[0], t[1], t[2], t[3]);
  a.sth2[i] = make_double2(t[4], t[5]);
  a.sth32[i] = make_float4((float)t[0], (float)t[1], (float)t[2], (float)t[3]);
  a.sth232[i] = make_float2((float)t[4], (float)t[5]);
}
// Polarizability of caller site c: s = abar^-1/2 (0 when not polarizable);
// writes the Thole factor and the polarizable flag of sorted site i.
__device__ __forceinline__ double rec_pol_of(const RecArgs& a, int i, int c) {
  const double* al = a.alpha + 6 * c;
  bool pol = false;
  for (int k = 0; k < 6; ++k) pol = pol || (al[k] != 0.0);
  const double abar = (al[0] + al[3] + al[5]) / 3.0;
  a.sa[i] = a.thole ? a.thole[c] : a.thole_default;
  a.is_pol[i] = pol ? 1 : 0;
  return pol && abar > 0.0 ? 1.0 / sqrt(abar) : 0.0;
}

__global__ void k_rec_mult(RecArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double q, d[3], t[6];
  rec_mult_of(a, a.perm[i], q, d, t);
  double4 p = a.sp[i];
  p.w = q;
  a.sp[i] = p;
  float4 p32 = a.sp32[i];
  p32.w = (float)q;
  a.sp32[i] = p32;
  double4 dd = a.sd[i];
  dd.x = d[0]; dd.y = d[1]; dd.z = d[2];
  a.sd[i] = dd;
  float4 dd32 = a.sd32[i];
  dd32.x = (float)d[0]; dd32.y = (float)d[1]; dd32.z = (float)d[2];
  a.sd32[i] = dd32;
  rec_mult_store(a, i, d, t);
}

// Polarizability records: s = abar^-1/2 (0 when not polarizable), Thole
// factor, polarizable flag.
__global__ void k_rec_pol(RecArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double s = rec_pol_of(a, i, a.perm[i]);
  double4 dd = a.sd[i];
  dd.w = s;
  a.sd[i] = dd;
  float4 dd32 = a.sd32[i];
  dd32.w = (float)s;
  a.sd32[i] = dd32;
}

// After a re-sort all three records change: one pass writes them whole.
__global__ void k_rec_all(RecArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int c = a.perm[i];
  double x[3], q, d[3], t[6];
  rec_pos_of(a, i, c, x);
  rec_mult_of(a, c, q, d, t);
  const double s = rec_pol_of(a, i, c);
  a.sp[i] = make_double4(x[0], x[1], x[2], q);
  a.sp32[i] = make_float4((float)x[0], (float)x[1], (float)x[2], (float)q);
  a.sd[i] = make_double4(d[0], d[1], d[2], s);
  a.sd32[i] = make_float4((float)d[0], (float)d[1], (float)d[2], (float)s);
  rec_mult_store(a, i, d, t);
}

// After the scan of is_pol: polarizable index maps and polarizable records,
// including alpha^-1 (checked symmetric positive definite).
__global__ void k_rec_polsites(RecArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const bool pol = a.is_pol[i] != 0;
  const int pi = a.pol_scan[i];
  a.polidx[i] = pol ? pi : -1;
  if (!pol) return;
  a.polsite[pi] = i;
  const int c = a.perm[i];
  const double4 p = a.sp[i];
  const double s = a.sd[i].w;
  a.pp[pi] = make_double4(p.x, p.y, p.z, s);
  a.pp32[pi] = make_float4((float)p.x, (float)p.y, (float)p.z, (float)s);
  a.pa[pi] = a.sa[i];
  const double* al = a.alpha + 6 * c;
  const double xx = al[0], xy = al[1], xz = al[2], yy = al[3], yz = al[4], zz = al[5];
  for (int k = 0; k < 6; ++k) a.alpha_s[6 * pi + k] = al[k];
  // Cholesky-type positivity test: leading principal minors > 0
  const double m1 = xx, m2 = xx * yy - xy * xy;
  const double det = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz);
  if (!(m1 > 0.0 && m2 > 0.0 && det > 0.0)) atomicOr(a.err, 4);
  const double id = 1.0 / det;
  a.ainv_s[6 * pi + 0] = (yy * zz - yz * yz) * id;
  a.ainv_s[6 * pi + 1] = (xz * yz - xy * zz) * id;
  a.ainv_s[6 * pi + 2] = (xy * yz - xz * yy) * id;
  a.ainv_s[6 * pi + 3] = (xx * zz - xz * xz) * id;
  a.ainv_s[6 * pi + 4] = (xy * xz - xx * yz) * id;
  a.ainv_s[6 * pi + 5] = (xx * yy - xy * xy) * id;
}

void launch_rec_all(const RecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_all, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}
void launch_rec_mult(const RecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_mult, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}
void launch_rec_pol(const RecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_pol, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}
void launch_rec_polsites(const RecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_polsites, dim3((a.n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
}

// Extremes over the polarizable sites: block maxima / minima combined with
// atomics on the IEEE bit patterns (order-preserving for non-negative
// doubles), so the result does not depend on block order.  out must hold
// 0 and +inf beforehand.
__global__ __launch_bounds__(kBlock) void k_pol_extents(RecArgs a, unsigned long long* out) {
  __shared__ double smax[kBlock], smin[kBlock];
  double amax = 0.0, tmin = INFINITY;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock) {
    if (!a.is_pol[i]) continue;
    const double s = a.sd[i].w;   // 1 / sqrt(mean polarizability)
    amax = fmax(amax, 1.0 / (s * s));
    tmin = fmin(tmin, fmax(a.sa[i], 0.0));
  }
  smax[threadIdx.x] = amax;
  smin[threadIdx.x] = tmin;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(smax[0]));
    atomicMin(&out[1], (unsigned long long)__double_as_longlong(smin[0]));
  }
}

void launch_pol_extents(const RecArgs& a, double* out, hipStream_t s) {
  unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
  // 0.0 and +inf
  launch_fill_int(reinterpret_cast<int*>(o), 0, 3, s);
  launch_fill_int(reinterpret_cast<int*>(o) + 3, 0x7ff00000, 1, s);
  int blocks = (a.n + kBlock - 1) / kBlock;
  blocks = blocks < 1 ? 1 : (blocks > 256 ? 256 : blocks);
  hipLaunchKernelGGL(k_pol_extents, dim3(blocks), dim3(kBlock), 0, s, a, o);
}

// ------------------------------------------------------------ neighbour lists
constexpr int kNlIB = 64;   // i-sites of a cell handled per pass (one per lane)

// The running count of each list for i-site t lives in lane t (cnt_*), read
// back wave-uniformly with readlane, so the inner loop needs neither LDS
// counters nor barriers; the block is a single wavefront.
__global__ __launch_bounds__(64) void k_nlist(NlistArgs a) {
  __shared__ double xi[kNlIB], yi[kNlIB], zi[kNlIB];
  __shared__ int moli[kNlIB], poli[kNlIB];
  const int lane = threadIdx.x;
  const int cell = blockIdx.x;
  const int cx = cell % a.nc[0];
  const int cy = (cell / a.nc[0]) % a.nc[1];
  const int cz = cell / (a.nc[0] * a.nc[1]);
  const int i0 = a.cell_start[cell], i1 = a.cell_start[cell + 1];
  const double L0 = a.box[0], L1 = a.box[1], L2 = a.box[2];
  const double iL0 = a.ibox[0], iL1 = a.ibox[1], iL2 = a.ibox[2];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // stencil extents per axis: all cells when the axis has fewer than 5
  int span[3], lo[3];
  const int c3[3] = {cx, cy, cz};
  for (int d = 0; d < 3; ++d) {
    if (a.nc[d] < 5) { span[d] = a.nc[d]; lo[d] = 0; }
    else { span[d] = 5; lo[d] = c3[d] - 2; }
  }
  int4 mx = make_int4(0, 0, 0, 0);   // the cell's count maxima
  for (int ib = i0; ib < i1; ib += kNlIB) {
    const int ni = min(kNlIB, i1 - ib);
    if (lane < ni) {
      const double4 p = a.sp[ib + lane];
      xi[lane] = p.x; yi[lane] = p.y; zi[lane] = p.z;
      moli[lane] = a.mol_s[ib + lane];
      poli[lane] = a.polidx[ib + lane];
    }
    __syncthreads();
    // counts of i-site `lane`: all near (cnt0) and far (cntf), in, pol, ipol
    int cnt0 = 0, cntf = 0, cnt1 = 0, cnt2 = 0, cnt3 = 0;
    for (int sz = 0; sz < span[2]; ++sz) {
      int zz = lo[2] + sz;
      zz = (zz + a.nc[2]) % a.nc[2];
      for (int sy = 0; sy < span[1]; ++sy) {
        int yy = lo[1] + sy;
        yy = (yy + a.nc[1]) % a.nc[1];
        const int rowcell = a.nc[0] * (yy + a.nc[1] * zz);
        // x cells of this row as at most two contiguous runs
        int rs[2], re[2], nrun;
        if (span[0] == a.nc[0]) {
          rs[0] = rowcell; re[0] = rowcell + a.nc[0]; nrun = 1;
        } else {
          const int x0 = lo[0], x1 = lo[0] + 4;
          if (x0 >= 0 && x1 < a.nc[0]) { rs[0] = rowcell + x0; re[0] = rowcell + x1 + 1; nrun = 1; }
          else if (x0 < 0) {
            rs[0] = rowcell; re[0] = rowcell + x1 + 1;
            rs[1] = rowcell + a.nc[0] + x0; re[1] = rowcell + a.nc[0]; nrun = 2;
          } else {
            rs[0] = rowcell + x0; re[0] = rowcell + a.nc[0];
            rs[1] = rowcell; re[1] = rowcell + (x1 - a.nc[0]) + 1; nrun = 2;
          }
        }
        for (int r = 0; r < nrun; ++r) {
          const int j0 = a.cell_start[rs[r]], j1 = a.cell_start[re[r]];
          for (int jc = j0; jc < j1; jc += 64) {
            const int j = jc + lane;
            const bool valid = j < j1;
            double xj = 0, yj = 0, zj = 0;
            int molj = -1, polj = -1;
            if (valid) {
              const double4 p = a.sp[j];
              xj = p.x; yj = p.y; zj = p.z;
              molj = a.mol_s[j];
              polj = a.polidx[j];
            }
            for (int t = 0; t < ni; ++t) {
              double dx = xi[t] - xj, dy = yi[t] - yj, dz = zi[t] - zj;
              if (a.periodic) {
                dx -= L0 * rint(dx * iL0);
                dy -= L1 * rint(dy * iL1);
                dz -= L2 * rint(dz * iL2);
              }
              const double r2 = dx * dx + dy * dy + dz * dz;
              const int i = ib + t;
              const int mi = moli[t], pi_ = poli[t];
              const bool same = valid && (molj == mi) && (j != i);
              const bool inter = valid && (molj != mi) && (r2 < a.cutoff2);
              const bool near = r2 < a.rsplit2;
              const bool pi = pi_ >= 0;
              const bool pj = polj >= 0;
              const unsigned long long b0 = __ballot(inter && near);
              const unsigned long long bf = __ballot(inter && !near);
              const unsigned long long b1 = __ballot(same);
              const unsigned long long b2 = __ballot(inter && pi && pj);
              const unsigned long long b3 = __ballot(same && pi && pj);
              const int base0 = __shfl(cnt0, t, 64), basef = __shfl(cntf, t, 64);
              const int base1 = __shfl(cnt1, t, 64);
              const int base2 = __shfl(cnt2, t, 64), base3 = __shfl(cnt3, t, 64);
              if (inter && near) {
                const int k = base0 + __popcll(b0 & below);
                if (k < a.cap_all) a.nb_all[(size_t)i * a.cap_all + k] = j;
              }
              if (inter && !near) {
                const int k = basef + __popcll(bf & below);
                if (k < a.cap_all) a.nb_all[(size_t)i * a.cap_all + a.cap_all - 1 - k] = j;
              }
              if (same) {
                const int k = base1 + __popcll(b1 & below);
                if (k < a.cap_in) a.nb_in[(size_t)i * a.cap_in + k] = j;
              }
              if (inter && pi && pj) {
                const int k = base2 + __popcll(b2 & below);
                if (k < a.cap_pol) a.nb_pol[(size_t)pi_ * a.cap_pol + k] = polj;
              }
              if (same && pi && pj) {
                const int k = base3 + __popcll(b3 & below);
                if (k < a.cap_ipol) a.nb_ipol[(size_t)pi_ * a.cap_ipol + k] = polj;
              }
              if (lane == t) {
                cnt0 += __popcll(b0);
                cntf += __popcll(bf);
                cnt1 += __popcll(b1);
                cnt2 += __popcll(b2);
                cnt3 += __popcll(b3);
              }
            }
          }
        }
      }
    }
    // counts, overflow maxima and the same-molecule completeness check
    if (lane < ni) {
      const int i = ib + lane;
      a.nc_all[i] = cnt0 + cntf;
      a.nc_near[i] = cnt0;
      a.nc_in[i] = cnt1;
      if (poli[lane] >= 0) {
        a.nc_pol[poli[lane]] = cnt2;
        a.nc_ipol[poli[lane]] = cnt3;
      }
      if (cnt1 != a.mol_count[moli[lane]] - 1) atomicOr(a.err, 1);
    }
    mx.x = max(mx.x, wave_max(lane < ni ? cnt0 + cntf : 0));
    mx.y = max(mx.y, wave_max(lane < ni ? cnt1 : 0));
    mx.z = max(mx.z, wave_max(lane < ni && poli[lane] >= 0 ? cnt2 : 0));
    mx.w = max(mx.w, wave_max(lane < ni && poli[lane] >= 0 ? cnt3 : 0));
    __syncthreads();
  }
  if (lane == 0) a.cellmax[cell] = mx;
}

// Periodic boxes with at least five cells along every axis.  Same lists, in
// the same order, as k_nlist, with changes that cut the work per candidate
// pair:
//  * the 5 x 5 rows of the stencil give at most 50 runs of consecutive
//    cells, each with a fixed periodic image shift (the stencil reaches a
//    wrapped cell through exactly one image), so a candidate's displacement
//    is x_i - (x_j + shift) without a per-pair rint;
//  * the runs are concatenated into one virtual candidate range, taken
//    kNlG chunks of 64 at a time into registers (a lane finds its run by
//    binary search over the run offsets), so chunks are full;
//  * each i-site's five running counts are read once per pass over those
//    chunks into wave-uniform (scalar) registers, so a candidate chunk costs
//    the distance test, the lane masks and the slot arithmetic of its hits;
//  * the cell's count maxima go to its own slot of cellmax (plain stores;
//    launch_cellmax_reduce folds them), not to one atomic per wavefront on
//    four shared addresses.
constexpr int kNlG = 4;   // candidate chunks per pass over the i-sites

__device__ __forceinline__ int rl(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
// lane masks straight from one vector compare (predicate codes of the
// compiler's compare intrinsics: ordered less-than; signed equal, >=)
constexpr int kCmpOLT = 4, kCmpEQ = 32, kCmpSGE = 39;
__device__ __forceinline__ unsigned long long mask_lt(double a, double b) {
  return __builtin_amdgcn_fcmp(a, b, kCmpOLT);
}
__device__ __forceinline__ unsigned long long mask_eq(int a, int b) {
  return __builtin_amdgcn_sicmp(a, b, kCmpEQ);
}

__global__ __launch_bounds__(64) void k_nlist_shift(NlistArgs a) {
  __shared__ double xi[kNlIB], yi[kNlIB], zi[kNlIB];
  __shared__ int run_s[50], run_off[51], run_code[50];
  const int lane = threadIdx.x;
  const int cell = blockIdx.x;
  const int nc0 = a.nc[0], nc1 = a.nc[1], nc2 = a.nc[2];
  const int cx = cell % nc0, cy = (cell / nc0) % nc1, cz = cell / (nc0 * nc1);
  const int i0 = a.cell_start[cell], i1 = a.cell_start[cell + 1];
  const double L0 = a.box[0], L1 = a.box[1], L2 = a.box[2];
  if (lane < 25) {
    const int dz = lane / 5 - 2, dy = lane % 5 - 2;
    int zz = cz + dz, zc = 1;
    if (zz < 0) { zz += nc2; zc = 0; } else if (zz >= nc2) { zz -= nc2; zc = 2; }
    int yy = cy + dy, yc = 1;
    if (yy < 0) { yy += nc1; yc = 0; } else if (yy >= nc1) { yy -= nc1; yc = 2; }
    const int row = nc0 * (yy + nc1 * zz);
    const int x0 = cx - 2, x1 = cx + 2;
    int f0, l0, c0, f1 = 0, l1 = -1, c1 = 1;   // cell ranges [f, l] and x image codes
    if (x0 >= 0 && x1 < nc0) { f0 = x0; l0 = x1; c0 = 1; }
    else if (x0 < 0) { f0 = 0; l0 = x1; c0 = 1; f1 = nc0 + x0; l1 = nc0 - 1; c1 = 0; }
    else { f0 = x0; l0 = nc0 - 1; c0 = 1; f1 = 0; l1 = x1 - nc0; c1 = 2; }
    const int yzc = 3 * yc + 9 * zc;
    run_s[2 * lane] = a.cell_start[row + f0];
    run_off[2 * lane + 1] = a.cell_start[row + l0 + 1] - a.cell_start[row + f0];
    run_code[2 * lane] = c0 + yzc;
    if (l1 >= f1) {
      run_s[2 * lane + 1] = a.cell_start[row + f1];
      run_off[2 * lane + 2] = a.cell_start[row + l1 + 1] - a.cell_start[row + f1];
    } else {
      run_s[2 * lane + 1] = 0;
      run_off[2 * lane + 2] = 0;
    }
    run_code[2 * lane + 1] = c1 + yzc;
  }
  __syncthreads();
  if (lane == 0) {
    run_off[0] = 0;
    for (int r = 1; r <= 50; ++r) run_off[r] += run_off[r - 1];
  }
  __syncthreads();
  const int ncand = run_off[50];
  const int cap_all = a.cap_all, cap_in = a.cap_in, cap_pol = a.cap_pol, cap_ipol = a.cap_ipol;
  const double cut2 = a.cutoff2, split2 = a.rsplit2;
  int4 mx = make_int4(0, 0, 0, 0);   // the cell's count maxima
  for (int ib = i0; ib < i1; ib += kNlIB) {
    const int ni = min(kNlIB, i1 - ib);
    // i-site `lane`: position in LDS (read back as a broadcast), molecule
    // and polarizable index in registers
    int mol_v = -1, pol_v = -1;
    if (lane < ni) {
      const double4 p = a.sp[ib + lane];
      xi[lane] = p.x; yi[lane] = p.y; zi[lane] = p.z;
      mol_v = a.mol_s[ib + lane];
      pol_v = a.polidx[ib + lane];
    }
    __syncthreads();
    // counts of i-site `lane`: all near (cnt0) and far (cntf), in, pol, ipol
    int cnt0 = 0, cntf = 0, cnt1 = 0, cnt2 = 0, cnt3 = 0;
    for (int c = 0; c < ncand; c += 64 * kNlG) {
      // a lane past the candidates sits far away in no molecule: it never
      // tests as a neighbour
      double xj[kNlG], yj[kNlG], zj[kNlG];
      int jj[kNlG], molj[kNlG], polj[kNlG];
      unsigned long long pjm[kNlG];
#pragma unroll
      for (int g = 0; g < kNlG; ++g) {
        const int cidx = c + g * 64 + lane;
        xj[g] = yj[g] = zj[g] = 1e30;
        jj[g] = -1; molj[g] = -1; polj[g] = -1;
        if (cidx < ncand) {
          int lo = 0, hi = 50;
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (run_off[mid] <= cidx) lo = mid; else hi = mid;
          }
          const int j = run_s[lo] + (cidx - run_off[lo]);
          const int code = run_code[lo];
          const double4 p = a.sp[j];
          xj[g] = p.x + L0 * (double)(code % 3 - 1);
          yj[g] = p.y + L1 * (double)((code / 3) % 3 - 1);
          zj[g] = p.z + L2 * (double)(code / 9 - 1);
          jj[g] = j;
          molj[g] = a.mol_s[j];
          polj[g] = a.polidx[j];
        }
        pjm[g] = __builtin_amdgcn_sicmp(polj[g], 0, kCmpSGE);
      }
      for (int t = 0; t < ni; ++t) {
        const double x = xi[t], y = yi[t], z = zi[t];
        const int i = ib + t;
        const int mi = rl(mol_v, t), pi_ = rl(pol_v, t);
        // site t's counts, wave-uniform for the chunks of this pass; a
        // lane's slot is the count plus the lower lanes of its mask
        int k0 = rl(cnt0, t), kf = rl(cntf, t), k1 = rl(cnt1, t), k2 = rl(cnt2, t),
            k3 = rl(cnt3, t);
        int* row_all = a.nb_all + (size_t)i * cap_all;
        int* row_in = a.nb_in + (size_t)i * cap_in;
        int* row_pol = a.nb_pol + (size_t)(pi_ >= 0 ? pi_ : 0) * cap_pol;
        int* row_ipol = a.nb_ipol + (size_t)(pi_ >= 0 ? pi_ : 0) * cap_ipol;
#pragma unroll
        for (int g = 0; g < kNlG; ++g) {
          const double dx = x - xj[g], dy = y - yj[g], dz = z - zj[g];
          const double r2 = dx * dx + dy * dy + dz * dz;
          // the same compares give the wave's masks and each lane's own
          // bit (the compiler folds them into one instruction each)
          const bool in_cut = r2 < cut2, in_mol = molj[g] == mi, in_near = r2 < split2;
          const unsigned long long bmol = mask_eq(molj[g], mi);
          const unsigned long long b0 = mask_lt(r2, cut2) & ~bmol;   // intermolecular
          if ((b0 | bmol) == 0ull) continue;   // no neighbour of site t in this chunk
          const bool inter = in_cut && !in_mol;
          const bool same = in_mol && jj[g] != i;
          unsigned long long b1 = 0ull;        // same molecule, not site t itself
          if (bmol) b1 = bmol & ~mask_eq(jj[g], i);
          if (b0) {
            const unsigned long long bnear = mask_lt(r2, split2);
            const unsigned long long bn = b0 & bnear, bf = b0 & ~bnear;
            if (bn) {
              if (inter && in_near) {
                const int k = lanes_below(bn, k0);
                if (k < cap_all) row_all[(unsigned)k] = jj[g];
              }
              k0 += __popcll(bn);
            }
            if (bf) {
              if (inter && !in_near) {
                const int k = lanes_below(bf, kf);
                if (k < cap_all) row_all[(unsigned)(cap_all - 1 - k)] = jj[g];
              }
              kf += __popcll(bf);
            }
          }
          if (b1) {
            if (same) {
              const int k = lanes_below(b1, k1);
              if (k < cap_in) row_in[(unsigned)k] = jj[g];
            }
            k1 += __popcll(b1);
          }
          if (pi_ >= 0) {
            const unsigned long long b2 = b0 & pjm[g], b3 = b1 & pjm[g];
            if (b2) {
              if (inter && polj[g] >= 0) {
                const int k = lanes_below(b2, k2);
                if (k < cap_pol) row_pol[(unsigned)k] = polj[g];
              }
              k2 += __popcll(b2);
            }
            if (b3) {
              if (same && polj[g] >= 0) {
                const int k = lanes_below(b3, k3);
                if (k < cap_ipol) row_ipol[(unsigned)k] = polj[g];
              }
              k3 += __popcll(b3);
            }
          }
        }
        if (lane == t) {
          cnt0 = k0; cntf = kf; cnt1 = k1; cnt2 = k2; cnt3 = k3;
        }
      }
    }
    if (lane < ni) {
      const int i = ib + lane;
      a.nc_all[i] = cnt0 + cntf;
      a.nc_near[i] = cnt0;
      a.nc_in[i] = cnt1;
      if (pol_v >= 0) {
        a.nc_pol[pol_v] = cnt2;
        a.nc_ipol[pol_v] = cnt3;
      }
      if (cnt1 != a.mol_count[mol_v] - 1) atomicOr(a.err, 1);
    }
    mx.x = max(mx.x, wave_max(lane < ni ? cnt0 + cntf : 0));
    mx.y = max(mx.y, wave_max(lane < ni ? cnt1 : 0));
    mx.z = max(mx.z, wave_max(pol_v >= 0 ? cnt2 : 0));
    mx.w = max(mx.w, wave_max(pol_v >= 0 ? cnt3 : 0));
    __syncthreads();
  }
  if (lane == 0) a.cellmax[cell] = mx;
}

__global__ __launch_bounds__(1024) void k_cellmax_reduce(const int4* cellmax, int ncell, int* out) {
  __shared__ int4 part[16];
  int4 m = make_int4(0, 0, 0, 0);
  for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
    const int4 v = cellmax[k];
    m.x = max(m.x, v.x); m.y = max(m.y, v.y); m.z = max(m.z, v.z); m.w = max(m.w, v.w);
  }
  m.x = wave_max(m.x); m.y = wave_max(m.y); m.z = wave_max(m.z); m.w = wave_max(m.w);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) part[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int4 r = part[0];
    for (int k = 1; k < nw; ++k) {
      r.x = max(r.x, part[k].x); r.y = max(r.y, part[k].y);
      r.z = max(r.z, part[k].z); r.w = max(r.w, part[k].w);
    }
    out[0] = r.x; out[1] = r.y; out[2] = r.z; out[3] = r.w;
  }
}

void launch_cellmax_reduce(const int4* cellmax, int ncell, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cellmax_reduce, dim3(1), dim3(1024), 0, s, cellmax, ncell, out);
}

void launch_nlist(const NlistArgs& a, int ncell, hipStream_t s) {
  if (a.periodic && a.nc[0] >= 5 && a.nc[1] >= 5 && a.nc[2] >= 5)
    hipLaunchKernelGGL(k_nlist_shift, dim3(ncell), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(k_nlist, dim3(ncell), dim3(64), 0, s, a);
}

}  // namespace sibfa
