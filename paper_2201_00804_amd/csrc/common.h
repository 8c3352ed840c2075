// Internal declarations shared by the library's translation units: device
// views of the cell-sorted system, small device helpers (wave and block
// reductions, minimum image, B-spline weights) and kernel launchers.
#pragma once
#include <initializer_list>
#include <utility>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sibfa {

constexpr double kCoulomb = 332.0637133;   // kcal*A/(mol*e^2)
constexpr double kDebye = 4.803204;        // D per e*A
constexpr double kSqrtPi = 1.7724538509055160273;
constexpr double kPi = 3.14159265358979323846;

constexpr int kBlock = 256;      // threads per block for site-parallel kernels
constexpr int kMaxOrder = 6;     // largest B-spline order supported

// Reduction slots (each has partials, a completion counter and a scalar).
enum Slot {
  S_EREAL = 0,   // real-space MM energy (e^2/A, times 1/2 applied)
  S_ESELF,       // Ewald self energy
  S_EREC,        // reciprocal energy of the last convolution
  S_PQ,          // p.Tp
  S_RZ0,         // r.z, ping
  S_RZ1,         // r.z, pong
  S_ZZ,          // z.z
  S_MUE,         // mu.E0
  S_MUTMU,       // mu.T mu
  S_AUX,         // real-space energy of same-molecule (excluded) pairs
  S_EREC0,       // reciprocal energy of the permanent multipoles
  S_EKIN,        // kinetic energy (molecular dynamics)
  S_EBOND,       // bond energy (molecular dynamics)
  S_EREP,        // stand-in repulsion energy (molecular dynamics)
  S_ECT,         // charge-transfer energy
  S_CTREC,       // reciprocal energy of the charge-transfer convolutions (unused)
  S_TCGD,        // dot products of the truncated-CG force pass
  // virial partials (written only when a virial is asked for), row-major
  // W_ab at slot + 3a + b unless noted
  S_VRI,                 // same-molecule pairs, 9 slots
  S_VRF = S_VRI + 9,     // intermolecular pairs, 9 slots
  S_VRK = S_VRF + 9,     // reciprocal m-space sum, 6 slots: xx yy zz xy xz yz
  S_VRG = S_VRK + 6,     // reciprocal site (amplitude) terms, 9 slots
  S_VRR = S_VRG + 9,     // rotation of local frames, 9 slots
  S_COUNT = S_VRR + 9
};

// Device view of the system in cell-sorted order.  Site records are AoS so
// that a neighbour gather touches one or two cache lines.
template <typename R>
struct Vec4 { using type = double4; };
template <>
struct Vec4<float> { using type = float4; };

struct SysView {
  int n, npol;
  int periodic;
  double box[3], ibox[3];
  double cutoff2;
  double beta;
  int uniform_thole;
  double thole_a;
  // sorted site records, FP64
  const double4* sp;    // x, y, z, q       (positions wrapped into the box)
  const double4* sd;    // dx, dy, dz, s    (s = abar^-1/2, 0 if not polarizable)
  const double4* sth;   // Theta xx, xy, xz, yy
  const double2* sth2;  // Theta yz, zz
  const double* sa;     // Thole factor per site
  const int* polidx;    // sorted site -> polarizable index, or -1
  // FP32 copies (mixed precision)
  const float4* sp32;
  const float4* sd32;
  const float4* sth32;
  const float2* sth232;
  // polarizable-site records (polarizable order = sorted order restricted)
  const int* polsite;   // polarizable index -> sorted site
  const double4* pp;    // x, y, z, s
  const float4* pp32;
  const double* pa;     // Thole factor
  const double* alpha;  // [npol][6] xx,xy,xz,yy,yz,zz
  const double* ainv;   // [npol][6]
  // neighbour lists (ELL: row i holds count[i] entries starting at i*cap)
  const int* nb_all;  const int* nc_all;  int cap_all;    // intermolecular, r < rc
  const int* nc_near;   // near pairs of the all list (see NlistArgs)
  const int* nb_in;   const int* nc_in;   int cap_in;     // same molecule
  const int* nb_pol;  const int* nc_pol;  int cap_pol;    // pol-pol, inter, r < rc
  const int* nb_ipol; const int* nc_ipol; int cap_ipol;   // pol-pol, same molecule
  // cached damped dipole-dipole coefficients (c1, c2) of the pol list (in
  // the context's precision) and of the same-molecule pol list (FP64)
  const double2* cpol;
  const float2* cpol32;
  const double2* cipol;
};

struct PmeView {
  int K[3];
  int order;
  int kxh;             // K[0]/2 + 1
  double scale[3];     // K_a / L_a
  double* Q;           // real spread grid [K2][K1][K0] (x fastest)
  double* phi;         // real potential grid, same layout
  double2* C;          // complex half grid [K2][K1][kxh]
  float* Q32;
  float* phi32;
  float2* C32;
  const double* G;     // influence function [K2][K1][kxh]
  const float* G32;
  const double2* tw[3];   // twiddles exp(-2 pi i k / K_a), k < K_a
  const float2* tw32[3];
  // FFT radices per axis, stage st in bits 2 st .. 2 st + 1 as radix - 2
  // (radices 2, 3, 4, 5), so the stage loop decodes them from a scalar
  int nrad[3];
  unsigned radcode[3];
  // spreading bricks: Bb[0] x Bb[1] x Bb[2] grid points per workgroup (each
  // <= kBrick; the last brick along an axis may be shorter but never below
  // order - 1 points), sites binned by the brick holding their base index
  int Bb[3];
  int nb[3];
  double* tiles;           // [nbricks][tile_size] spreading tiles
  float* tiles32;
  int tile_size;           // (Bb0 + p - 1)(Bb1 + p - 1)(Bb2 + p - 1)
  const int* bstart_pol;   // [nbricks + 1]
  const int* border_pol;   // polarizable indices grouped by brick
  const int* bstart_all;
  const int* border_all;   // sorted-site indices grouped by brick
  const int* stop;         // see Reduce::stop
  int erec_slot;           // reduction slot of the convolution's E_rec partials
  double beta;             // Ewald parameter (the virial's m-space weights)
};

constexpr int kBrick = 8;

// Spreading tiles (see the spreading kernels): the grid value at (gx, gy,
// gz) is the sum, in a fixed order, of the entries of the tiles that cover
// it -- its own brick's and, along each axis where it lies within order - 1
// points of the next brick, that brick's.
template <typename T>
__device__ __forceinline__ const T* tile_data(const PmeView& pm);
template <>
__device__ __forceinline__ const double* tile_data<double>(const PmeView& pm) { return pm.tiles; }
template <>
__device__ __forceinline__ const float* tile_data<float>(const PmeView& pm) { return pm.tiles32; }

template <typename T>
__device__ __forceinline__ T fold_point(const PmeView& pm, int gx, int gy, int gz) {
  const int P = pm.order;
  const int g[3] = {gx, gy, gz};
  int bi[3][2], ti[3][2], nd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int B = pm.Bb[a], b = g[a] / B, ox = g[a] - b * B;
    const int Bs = min(B, pm.K[a] - b * B);
    bi[a][0] = b;
    ti[a][0] = ox + P - 1;
    bi[a][1] = b + 1 < pm.nb[a] ? b + 1 : 0;
    ti[a][1] = ox - Bs + P - 1;
    nd[a] = ti[a][1] >= 0 ? 2 : 1;
  }
  const int T0 = pm.Bb[0] + P - 1, T1 = pm.Bb[1] + P - 1;
  const T* tiles = tile_data<T>(pm);
  // all (up to eight) loads issued before the first add
  T v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
    v[k] = T(0);
    if (dx < nd[0] && dy < nd[1] && dz < nd[2]) {
      const int bb = bi[0][dx] + pm.nb[0] * (bi[1][dy] + pm.nb[1] * bi[2][dz]);
      v[k] = tiles[(size_t)bb * pm.tile_size + (ti[2][dz] * T1 + ti[1][dy]) * T0 + ti[0][dx]];
    }
  }
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if ((k & 1) < nd[0] && ((k >> 1) & 1) < nd[1] && (k >> 2) < nd[2]) sum += v[k];
  return sum;
}

// Grid base index of a coordinate along one axis: floor(x K / L) wrapped
// into [0, K), and the fractional offset.
__device__ __forceinline__ int grid_base(double x, double scale, int K, double* frac) {
  const double u = x * scale;
  const double fl = floor(u);
  // positions arrive wrapped into the box; the clamp and the modulo keep
  // any other value in [0, K) as well
  int k = (int)fmin(fmax(fl, -1073741824.0), 1073741824.0);
  if (k >= K || k < 0) {
    k %= K;
    if (k < 0) k += K;
  }
  *frac = u - fl;
  return k;
}

// Deterministic reductions without device-wide fences: a producing kernel
// writes one partial sum per block (block_partial); whoever needs the total
// -- a later kernel (slot_total, every block summing the same partials in
// the same order) or the host -- adds the partials in index order.  The
// host records how many partials each slot's last producer wrote.
struct Reduce {
  double* partials;      // [S_COUNT][max_blocks]
  int max_blocks;
  int nparts[S_COUNT];
  const int* stop;       // solver iterations: kernels return at once when *stop != 0
};

__device__ __forceinline__ bool stopped(const int* stop) { return stop && *stop; }

// ---------------------------------------------------------------- helpers
// Workgroups are dealt to the GPU's XCDs round robin (blockIdx % kXcd), and
// each XCD has its own L2.  Site-parallel kernels over the cell-sorted order
// map the launch index so that each XCD processes one contiguous, spatially
// compact range of sites: the neighbours it gathers then stay in its L2.
// The map is a bijection of [0, gridDim.x) for any grid size.
constexpr int kXcd = 8;
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int x = b % kXcd, per = nb / kXcd, extra = nb % kXcd;
  return x * per + (x < extra ? x : extra) + b / kXcd;
}
// For every active lane, adds 1 to base[key], with one atomic per distinct
// key of the wavefront (sorted or clustered keys make that a few atomics
// instead of one per lane on the same address); returns the lane's slot,
// the counter's old value plus the number of lower active lanes with the
// same key.  Every lane of the wavefront must call it.
__device__ __forceinline__ int wave_atomic_inc(int* base, int key, bool active) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long todo = __ballot(active);
  int slot = 0;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int k = __shfl(key, leader, 64);
    const unsigned long long same = __ballot(active && key == k);
    int old = 0;
    if (lane == leader) old = atomicAdd(&base[k], __popcll(same));
    old = __shfl(old, leader, 64);
    if (active && key == k) slot = old + __popcll(same & below);
    todo &= ~same;
  }
  return slot;
}
// base + the number of set bits of mask below this lane
__device__ __forceinline__ int lanes_below(unsigned long long mask, int base) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)mask, (unsigned)base));
}

// Orders this wave's LDS accesses before the call against those after it
// (the lanes of a wave issue together, so no hardware barrier is needed;
// this keeps the compiler from moving LDS loads and stores across it).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over groups of G consecutive lanes (G a power of two <= 64).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Block sum of v written as this block's partial of the slot.  Every thread
// of the block must call it (blockDim.x <= kBlock).
__device__ __forceinline__ void block_partial(double v, const Reduce& red, int slot) {
  __shared__ double sh[kBlock / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    red.partials[(size_t)slot * red.max_blocks + blockIdx.x] = s;
  }
  __syncthreads();
}

// Total of a slot written by an earlier kernel, returned to every thread.
// Every thread of the block must call it.
__device__ __forceinline__ double slot_total(const Reduce& red, int slot) {
  __shared__ double sh[kBlock / 64];
  const int n = red.nparts[slot];
  double v = 0.0;
  for (int b = threadIdx.x; b < n; b += blockDim.x)
    v += red.partials[(size_t)slot * red.max_blocks + b];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  __syncthreads();
  return s;
}

template <typename R>
__device__ __forceinline__ R min_image(R d, R L, R iL) {
  return d - L * rint(d * iL);
}

// Cardinal B-spline weights of order P at fractional offset w in [0,1):
// th[D][t] is the D-th derivative of M_P(w + t) for t = 0..P-1, grid point
// index floor(u) - t.  Built with the two-term recursion
//   M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)) / (n - 1)
// and derivatives from differences of lower orders.
template <typename R, int P, int ND>
__device__ __forceinline__ void bspline_weights(R w, R th[ND + 1][P]) {
  R lev[P][P];   // lev[k][t] = M_{k+1}(w + t)
  lev[0][0] = R(1);
#pragma unroll
  for (int t = 1; t < P; ++t) lev[0][t] = R(0);
#pragma unroll
  for (int k = 1; k < P; ++k) {
    const int n = k + 1;
    const R inv = R(1) / R(n - 1);
#pragma unroll
    for (int t = P - 1; t >= 0; --t) {
      const R u = w + R(t);
      const R a = (t <= k - 1) ? lev[k - 1][t] : R(0);
      const R b = (t >= 1 && t - 1 <= k - 1) ? lev[k - 1][t - 1] : R(0);
      lev[k][t] = (u * a + (R(n) - u) * b) * inv;
    }
  }
#pragma unroll
  for (int t = 0; t < P; ++t) th[0][t] = lev[P - 1][t];
  if (ND >= 1) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const R a = lev[P - 2][t];
      const R b = (t >= 1) ? lev[P - 2][t - 1] : R(0);
      th[ND >= 1 ? 1 : 0][t] = a - b;
    }
  }
  if (ND >= 2) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const R a = lev[P - 3][t];
      const R b = (t >= 1) ? lev[P - 3][t - 1] : R(0);
      const R c = (t >= 2) ? lev[P - 3][t - 2] : R(0);
      th[ND >= 2 ? 2 : 0][t] = a - R(2) * b + c;
    }
  }
  if (ND >= 3) {
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const R a = lev[P - 4][t];
      const R b = (t >= 1) ? lev[P - 4][t - 1] : R(0);
      const R c = (t >= 2) ? lev[P - 4][t - 2] : R(0);
      const R d = (t >= 3) ? lev[P - 4][t - 3] : R(0);
      th[ND >= 3 ? 3 : 0][t] = a - R(3) * b + R(3) * c - d;
    }
  }
}

// Grid base indices and B-spline weights (derivatives up to ND) of a site
// along the three axes.
template <typename R, int P, int ND>
__device__ __forceinline__ void site_splines(const PmeView& pm, double x, double y, double z,
                                             int base[3], R th[3][ND + 1][P]) {
  const double xs[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double fr;
    base[a] = grid_base(xs[a], pm.scale[a], pm.K[a], &fr);
    bspline_weights<R, P, ND>((R)fr, th[a]);
  }
}

// ---------------------------------------------------------------- launchers
// nlist.hip
void launch_fill_int(int* p, int v, size_t n, hipStream_t s);
constexpr int kFillMax = 8;
struct FillList {
  int n;
  int* p[kFillMax];
  size_t cnt[kFillMax];
  int v;
};
// every (buffer, count) set to v, in one launch per eight buffers
void launch_fill_ints(std::initializer_list<std::pair<int*, size_t>> bufs, int v, hipStream_t s);
void launch_fill_double(double* p, double v, size_t n, hipStream_t s);
void launch_fill_float(float* p, float v, size_t n, hipStream_t s);
size_t scan_temp_ints(int n);
void launch_exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t s);

}  // namespace sibfa
