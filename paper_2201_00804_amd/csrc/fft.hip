// 3D FFT convolution of the PME grid, written for LDS.
//
// phi = IFFT3( G * FFT3(Q) ) over a real K0 x K1 x K2 grid (x fastest),
// with the half spectrum kx = 0..K0/2 kept after the real-to-complex x pass.
// Five passes, each a kernel in which one workgroup loads a batch of lines
// into LDS, transforms them there and writes them back:
//   x  r2c        rows of Q -> half-spectrum rows
//   y  forward    lines along y, a block of consecutive kx per workgroup so
//                 global accesses stay coalesced
//   z  forward, multiply by G (and accumulate E_rec = 1/2 sum G |F|^2 over
//      the full spectrum), z inverse -- fused, the z lines never leave LDS
//   y  inverse
//   x  c2r        Hermitian completion of the row, inverse, real part -> phi
// The inverse is unnormalised: phi(k) = sum_m G(m) F(m) exp(+2 pi i m.k/K).
//
// Line transforms are mixed-radix Stockham autosort (radices 4, 2, 3, 5),
// ping-ponging between two LDS buffers; twiddles come from a per-axis table
// exp(-2 pi i k/K_a), conjugated for the inverse.
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "kernels.h"

namespace sibfa {

constexpr size_t kPlaneLdsMax = 160 * 1024;   // LDS a gfx950 workgroup may use

template <typename T> struct CT;
template <> struct CT<double> { using type = double2; };
template <> struct CT<float> { using type = float2; };

template <typename T>
using cplx = typename CT<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  cplx<T> r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { cplx<T> r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { cplx<T> r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
// multiply by -i (forward) or +i (inverse): sgn = -1 forward, +1 inverse
template <typename T>
__device__ __forceinline__ cplx<T> cmuli(cplx<T> a, T sgn) { cplx<T> r; r.x = -sgn * a.y; r.y = sgn * a.x; return r; }
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { cplx<T> r; r.x = a.x * s; r.y = a.y * s; return r; }

// In-place small DFT of v[0..R-1]; sgn = -1 forward, +1 inverse.
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T>* v, T sgn) {
  if (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
  } else if (R == 4) {
    const cplx<T> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    const cplx<T> s02 = cadd<T>(a0, a2), d02 = csub<T>(a0, a2);
    const cplx<T> s13 = cadd<T>(a1, a3), d13 = cmuli<T>(csub<T>(a1, a3), sgn);
    v[0] = cadd<T>(s02, s13);
    v[2] = csub<T>(s02, s13);
    v[1] = cadd<T>(d02, d13);
    v[3] = csub<T>(d02, d13);
  } else if (R == 3) {
    const T c = T(-0.5), s = T(0.86602540378443864676);
    const cplx<T> a0 = v[0], a1 = v[1], a2 = v[2];
    const cplx<T> t = cadd<T>(a1, a2);
    const cplx<T> m = cadd<T>(a0, cscale<T>(t, c));
    const cplx<T> d = cmuli<T>(csub<T>(a1, a2), sgn * s);
    v[0] = cadd<T>(a0, t);
    v[1] = cadd<T>(m, d);
    v[2] = csub<T>(m, d);
  } else if (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    const cplx<T> a0 = v[0];
    const cplx<T> b1 = cadd<T>(v[1], v[4]), b2 = cadd<T>(v[2], v[3]);
    const cplx<T> d1 = csub<T>(v[1], v[4]), d2 = csub<T>(v[2], v[3]);
    const cplx<T> m1 = cadd<T>(a0, cadd<T>(cscale<T>(b1, c1), cscale<T>(b2, c2)));
    const cplx<T> m2 = cadd<T>(a0, cadd<T>(cscale<T>(b1, c2), cscale<T>(b2, c1)));
    const cplx<T> n1 = cmuli<T>(cadd<T>(cscale<T>(d1, s1), cscale<T>(d2, s2)), sgn);
    const cplx<T> n2 = cmuli<T>(csub<T>(cscale<T>(d1, s2), cscale<T>(d2, s1)), sgn);
    v[0] = cadd<T>(a0, cadd<T>(b1, b2));
    v[1] = cadd<T>(m1, n1);
    v[4] = csub<T>(m1, n1);
    v[2] = cadd<T>(m2, n2);
    v[3] = csub<T>(m2, n2);
  }
}

// ---- workgroup-level helpers.  NT is the workgroup size, a constant, so
// that no loop re-reads the block size after a barrier.

// f(i, j) over [0, I) x [0, J), j fastest across threads.
template <int NT, typename F>
__device__ __forceinline__ void for2d(int I, int J, F f) {
  if (J <= NT) {
    const int is = NT / J, j = threadIdx.x % J, i0 = threadIdx.x / J;
    if (i0 < is)
      for (int i = i0; i < I; i += is) f(i, j);
  } else {
    for (int i = 0; i < I; ++i)
      for (int j = threadIdx.x; j < J; j += NT) f(i, j);
  }
}

// The same traversal with up to kLoadU loads in flight per thread:
// v = ld(i, j), then st(i, j, v).
constexpr int kLoadU = 6;
template <int NT, typename V, typename LD, typename ST>
__device__ __forceinline__ void stage2d(int I, int J, LD ld, ST st) {
  if (J <= NT) {
    const int is = NT / J, j = threadIdx.x % J, i0 = threadIdx.x / J;
    if (i0 >= is) return;
    for (int ib = i0; ib < I; ib += kLoadU * is) {
      V v[kLoadU];
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        const int i = ib + u * is;
        if (i < I) v[u] = ld(i, j);
      }
#pragma unroll
      for (int u = 0; u < kLoadU; ++u) {
        const int i = ib + u * is;
        if (i < I) st(i, j, v[u]);
      }
    }
  } else {
    for (int i = 0; i < I; ++i)
      for (int jb = threadIdx.x; jb < J; jb += kLoadU * NT) {
        V v[kLoadU];
#pragma unroll
        for (int u = 0; u < kLoadU; ++u) {
          const int j = jb + u * NT;
          if (j < J) v[u] = ld(i, j);
        }
#pragma unroll
        for (int u = 0; u < kLoadU; ++u) {
          const int j = jb + u * NT;
          if (j < J) st(i, j, v[u]);
        }
      }
  }
}

// One Stockham stage of radix R on one line (src, dst already offset to
// the line), butterflies j = lt, lt + tpl, ... < N / R.  Ns (the product of
// the earlier radices) is a power of two until the first radix 3 or 5, so
// the index split is a shift and a mask for most stages.
template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cplx<T>* src, cplx<T>* dst, int N, int Ns,
                                               int lt, int tpl, const cplx<T>* tw, T sgn) {
  const int nb = N / R;
  const int twstep = N / (Ns * R);
  const bool p2 = (Ns & (Ns - 1)) == 0;
  const int sh = __builtin_ctz((unsigned)Ns);
  for (int j = lt; j < nb; j += tpl) {
    int q, k;
    if (p2) {
      q = j >> sh;
      k = j & (Ns - 1);
    } else {
      q = j / Ns;
      k = j - q * Ns;
    }
    const int kt = k * twstep;   // twiddle index k r twstep < N (k < Ns, r < R)
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx<T> a = src[j + r * nb];
      if (r > 0 && Ns > 1) {
        cplx<T> w = tw[kt * r];
        w.y *= -sgn;   // table holds exp(-2 pi i m/N); inverse uses the conjugate
        a = cmul<T>(a, w);
      }
      v[r] = a;
    }
    dft_small<T, R>(v, sgn);
    const int o = q * (Ns * R) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * Ns] = v[r];
  }
}

// Transform nl <= NT lines of length N, line stride ls, held in a (scratch
// b); returns the buffer holding the result.  Each line is served by a
// fixed group of NT / nl threads.  Every thread of the block must call it.
template <typename T, int NT>
__device__ cplx<T>* lds_fft(cplx<T>* a, cplx<T>* b, int N, int nl, int ls, unsigned radcode,
                            int nrad, const cplx<T>* tw, T sgn) {
  const int tpl = NT / nl;
  const int line = threadIdx.x / tpl, lt = threadIdx.x - line * tpl;
  const bool act = line < nl;
  const int off = line * ls;
  int Ns = 1;
  cplx<T>* in = a;
  cplx<T>* out = b;
  for (int st = 0; st < nrad; ++st) {
    __syncthreads();
    const int R = 2 + (int)((radcode >> (2 * st)) & 3u);
    if (act) {
      if (R == 4) stockham_stage<T, 4>(in + off, out + off, N, Ns, lt, tpl, tw, sgn);
      else if (R == 2) stockham_stage<T, 2>(in + off, out + off, N, Ns, lt, tpl, tw, sgn);
      else if (R == 3) stockham_stage<T, 3>(in + off, out + off, N, Ns, lt, tpl, tw, sgn);
      else stockham_stage<T, 5>(in + off, out + off, N, Ns, lt, tpl, tw, sgn);
    }
    Ns *= R;
    cplx<T>* t = in; in = out; out = t;
  }
  __syncthreads();
  return in;
}

// Copies the axis' twiddle table into LDS (after the two line buffers);
// the caller's first barrier (inside lds_fft) orders it before use.
template <typename T, int NT>
__device__ __forceinline__ const cplx<T>* stage_twiddles(const cplx<T>* src, cplx<T>* dst, int N) {
  for (int k = threadIdx.x; k < N; k += NT) dst[k] = src[k];
  return dst;
}

template <typename T> __device__ __forceinline__ T* gQ(const PmeView& pm);
template <> __device__ __forceinline__ double* gQ<double>(const PmeView& pm) { return pm.Q; }
template <> __device__ __forceinline__ float* gQ<float>(const PmeView& pm) { return pm.Q32; }
template <typename T> __device__ __forceinline__ T* gPhi(const PmeView& pm);
template <> __device__ __forceinline__ double* gPhi<double>(const PmeView& pm) { return pm.phi; }
template <> __device__ __forceinline__ float* gPhi<float>(const PmeView& pm) { return pm.phi32; }
template <typename T> __device__ __forceinline__ cplx<T>* gC(const PmeView& pm);
template <> __device__ __forceinline__ double2* gC<double>(const PmeView& pm) { return pm.C; }
template <> __device__ __forceinline__ float2* gC<float>(const PmeView& pm) { return pm.C32; }
template <typename T> __device__ __forceinline__ const cplx<T>* gTw(const PmeView& pm, int a);
template <> __device__ __forceinline__ const double2* gTw<double>(const PmeView& pm, int a) { return pm.tw[a]; }
template <> __device__ __forceinline__ const float2* gTw<float>(const PmeView& pm, int a) { return pm.tw32[a]; }
template <typename T> __device__ __forceinline__ const T* gG(const PmeView& pm);
template <> __device__ __forceinline__ const double* gG<double>(const PmeView& pm) { return pm.G; }
template <> __device__ __forceinline__ const float* gG<float>(const PmeView& pm) { return pm.G32; }

// LDS line buffers use a stride of length + 1 (an odd number of complex
// values), so lines handled side by side in a wave fall in different banks.

// ---- x pass, real to half complex.  Block: nl rows.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_x_r2c(PmeView pm, int nl) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[0], ls = N + 1, h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nl * ls;
  const int nrows = pm.K[1] * pm.K[2];
  const int row0 = blockIdx.x * nl;
  const int rows = min(nl, nrows - row0);
  const T* Q = gQ<T>(pm);
  stage2d<kBlock, cplx<T>>(nl, N, [&](int l, int x) {
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (l < rows) v.x = Q[(size_t)(row0 + l) * N + x];
    return v;
  }, [&](int l, int x, cplx<T> v) { a[l * ls + x] = v; });
  const cplx<T>* tw = stage_twiddles<T, kBlock>(gTw<T>(pm, 0), b + nl * ls, N);
  cplx<T>* res = lds_fft<T, kBlock>(a, b, N, nl, ls, pm.radcode[0], pm.nrad[0], tw, T(-1));
  cplx<T>* C = gC<T>(pm);
  for2d<kBlock>(nl, h, [&](int l, int k) {
    if (l < rows) C[(size_t)(row0 + l) * h + k] = res[l * ls + k];
  });
}

// ---- y pass (both directions).  Block: (z, block of nb consecutive kx).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_y(PmeView pm, int nb, T sgn) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[1], ls = N + 1, h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nb * ls;
  const int nkb = (h + nb - 1) / nb;
  const int z = blockIdx.x / nkb;
  const int kx0 = (blockIdx.x - z * nkb) * nb;
  const int cols = min(nb, h - kx0);
  cplx<T>* C = gC<T>(pm);
  stage2d<kBlock, cplx<T>>(N, nb, [&](int y, int c) {
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (c < cols) v = C[((size_t)z * N + y) * h + kx0 + c];
    return v;
  }, [&](int y, int c, cplx<T> v) { a[c * ls + y] = v; });
  const cplx<T>* tw = stage_twiddles<T, kBlock>(gTw<T>(pm, 1), b + nb * ls, N);
  cplx<T>* res = lds_fft<T, kBlock>(a, b, N, nb, ls, pm.radcode[1], pm.nrad[1], tw, sgn);
  for2d<kBlock>(N, nb, [&](int y, int c) {
    if (c < cols) C[((size_t)z * N + y) * h + kx0 + c] = res[c * ls + y];
  });
}

// ---- z pass: forward, influence function, inverse.  Block: (y, kx block).
// VIR: also the m-space sum of the reciprocal virial,
//   sum_m G(m) (pi^2/beta^2 + 1/m^2) m_a m_b |FFT(Q)(m)|^2
// over the full spectrum (the half spectrum with the same weights as the
// energy), with m_a = f_a / L_a and f_a the signed frequency of the index
// (an index at K/2 taken as -K/2).
template <typename T, bool VIR>
__global__ __launch_bounds__(kBlock) void k_fft_z_conv(PmeView pm, Reduce red, int nb) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[2], ls = N + 1, K1 = pm.K[1], h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nb * ls;
  const int nkb = (h + nb - 1) / nb;
  const int y = blockIdx.x / nkb;
  const int kx0 = (blockIdx.x - y * nkb) * nb;
  const int cols = min(nb, h - kx0);
  cplx<T>* C = gC<T>(pm);
  const T* G = gG<T>(pm);
  // this thread's (z, c) in the multiply step (nb <= kBlock); its first
  // influence-function values are fetched while the forward transform runs
  const int zs = kBlock / nb, cth = threadIdx.x % nb, z0 = threadIdx.x / nb;
  const bool mact = z0 < zs && cth < cols;
  T gpre[kLoadU];
#pragma unroll
  for (int u = 0; u < kLoadU; ++u) {
    const int z = z0 + u * zs;
    gpre[u] = (mact && z < N) ? G[((size_t)z * K1 + y) * h + kx0 + cth] : T(0);
  }
  stage2d<kBlock, cplx<T>>(N, nb, [&](int z, int c) {
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (c < cols) v = C[((size_t)z * K1 + y) * h + kx0 + c];
    return v;
  }, [&](int z, int c, cplx<T> v) { a[c * ls + z] = v; });
  const cplx<T>* tw = stage_twiddles<T, kBlock>(gTw<T>(pm, 2), b + nb * ls, N);
  cplx<T>* res = lds_fft<T, kBlock>(a, b, N, nb, ls, pm.radcode[2], pm.nrad[2], tw, T(-1));
  double e_part = 0.0;
  double vk[6] = {0, 0, 0, 0, 0, 0};
  if (mact) {
    const int kx = kx0 + cth;
    const double mult = (kx == 0 || 2 * kx == pm.K[0]) ? 1.0 : 2.0;
    double mx = 0.0, my = 0.0, b2 = 0.0;
    if (VIR) {
      const int fx = 2 * kx == pm.K[0] ? -kx : kx;
      const int fy = 2 * y < pm.K[1] ? y : y - pm.K[1];
      mx = fx * pm.scale[0] / pm.K[0];
      my = fy * pm.scale[1] / pm.K[1];
      b2 = kPi * kPi / (pm.beta * pm.beta);
    }
    auto apply = [&](int z, T g) {
      cplx<T> v = res[cth * ls + z];
      const double a2 = (double)v.x * v.x + (double)v.y * v.y;
      e_part += 0.5 * mult * (double)g * a2;
      if (VIR) {
        const int fz = 2 * z < N ? z : z - N;
        const double mz = fz * pm.scale[2] / N;
        const double m2 = mx * mx + my * my + mz * mz;
        if (m2 > 0.0) {
          const double w = mult * (double)g * a2 * (b2 + 1.0 / m2);
          vk[0] += w * mx * mx; vk[1] += w * my * my; vk[2] += w * mz * mz;
          vk[3] += w * mx * my; vk[4] += w * mx * mz; vk[5] += w * my * mz;
        }
      }
      v.x *= g; v.y *= g;
      res[cth * ls + z] = v;
    };
#pragma unroll
    for (int u = 0; u < kLoadU; ++u) {
      const int z = z0 + u * zs;
      if (z < N) apply(z, gpre[u]);
    }
    for (int z = z0 + kLoadU * zs; z < N; z += zs) apply(z, G[((size_t)z * K1 + y) * h + kx]);
  }
  cplx<T>* other = (res == a) ? b : a;
  cplx<T>* res2 = lds_fft<T, kBlock>(res, other, N, nb, ls, pm.radcode[2], pm.nrad[2], tw, T(1));
  for2d<kBlock>(N, nb, [&](int z, int c) {
    if (c < cols) C[((size_t)z * K1 + y) * h + kx0 + c] = res2[c * ls + z];
  });
  block_partial(e_part, red, pm.erec_slot);
  if (VIR)
#pragma unroll
    for (int k = 0; k < 6; ++k) block_partial(vk[k], red, S_VRK + k);
}

// ---- x pass, half complex to real.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_x_c2r(PmeView pm, int nl) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[0], ls = N + 1, h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nl * ls;
  const int nrows = pm.K[1] * pm.K[2];
  const int row0 = blockIdx.x * nl;
  const int rows = min(nl, nrows - row0);
  const cplx<T>* C = gC<T>(pm);
  stage2d<kBlock, cplx<T>>(nl, N, [&](int l, int k) {
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (l < rows) {
      const size_t rb = (size_t)(row0 + l) * h;
      if (k < h) v = C[rb + k];
      else {
        v = C[rb + (N - k)];
        v.y = -v.y;
      }
    }
    return v;
  }, [&](int l, int k, cplx<T> v) { a[l * ls + k] = v; });
  const cplx<T>* tw = stage_twiddles<T, kBlock>(gTw<T>(pm, 0), b + nl * ls, N);
  cplx<T>* res = lds_fft<T, kBlock>(a, b, N, nl, ls, pm.radcode[0], pm.nrad[0], tw, T(1));
  T* phi = gPhi<T>(pm);
  for2d<kBlock>(nl, N, [&](int l, int x) {
    if (l < rows) phi[(size_t)(row0 + l) * N + x] = res[l * ls + x].x;
  });
}

// ---- whole z-planes in LDS (grids whose planes fit in a workgroup's LDS)
// Forward: transform pairs of real rows of Q (folded from the spreading
// tiles by k_spread_fold) as one complex line (rows y and y + 1 as real and
// imaginary parts), split them into the two half spectra, then transform
// the columns (one per kx) along y; writes C[z][y][kx].
// Inverse: columns along y, then pairs of Hermitian-completed rows combined
// as X + iY into one complex line, inverse, real and imaginary parts ->
// rows y and y + 1 of phi.  The imaginary parts of the kx = 0 and kx = K0/2
// entries are dropped, as a real inverse does.
// 512 threads (two waves per SIMD): small enough that a plane workgroup
// finds room on a CU beside the waves of the real-space matvec, which runs
// on the other stream at the same time (1024-thread planes waited for the
// matvec to drain; 256 threads leave the plane itself too slow).
constexpr int kPlaneThreads = 512;

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_fft_plane_fwd(PmeView pm) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh, z = blockIdx.x;
  const int rs = K0 + 1, cs = K1 + 1;           // row and column strides
  const int bufsz = max((K1 / 2) * rs, h * cs);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + bufsz;
  cplx<T>* tw0 = B + bufsz;
  cplx<T>* tw1 = tw0 + K0;
  stage_twiddles<T, NT>(gTw<T>(pm, 0), tw0, K0);
  stage_twiddles<T, NT>(gTw<T>(pm, 1), tw1, K1);
  const T* Q = gQ<T>(pm) + (size_t)z * K1 * K0;
  stage2d<NT, cplx<T>>(K1 / 2, K0, [&](int m, int x) {
    cplx<T> v;
    v.x = Q[(2 * m) * K0 + x];
    v.y = Q[(2 * m + 1) * K0 + x];
    return v;
  }, [&](int m, int x, cplx<T> v) { A[m * rs + x] = v; });
  cplx<T>* rows = lds_fft<T, NT>(A, B, K0, K1 / 2, rs, pm.radcode[0], pm.nrad[0], tw0, T(-1));
  cplx<T>* cols = rows == A ? B : A;
  for2d<NT>(K1 / 2, h, [&](int m, int k) {
    const cplx<T> zk = rows[m * rs + k];
    const cplx<T> zn = rows[m * rs + (k == 0 ? 0 : K0 - k)];
    cplx<T> X, Y;
    X.x = T(0.5) * (zk.x + zn.x);
    X.y = T(0.5) * (zk.y - zn.y);
    Y.x = T(0.5) * (zk.y + zn.y);
    Y.y = T(0.5) * (zn.x - zk.x);
    cols[k * cs + 2 * m] = X;
    cols[k * cs + 2 * m + 1] = Y;
  });
  cplx<T>* res = lds_fft<T, NT>(cols, rows, K1, h, cs, pm.radcode[1], pm.nrad[1], tw1, T(-1));
  cplx<T>* C = gC<T>(pm) + (size_t)z * K1 * h;
  for2d<NT>(K1, h, [&](int y, int k) { C[y * h + k] = res[k * cs + y]; });
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_fft_plane_inv(PmeView pm) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh, z = blockIdx.x;
  const int rs = K0 + 1, cs = K1 + 1;
  const int bufsz = max((K1 / 2) * rs, h * cs);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + bufsz;
  cplx<T>* tw0 = B + bufsz;
  cplx<T>* tw1 = tw0 + K0;
  stage_twiddles<T, NT>(gTw<T>(pm, 0), tw0, K0);
  stage_twiddles<T, NT>(gTw<T>(pm, 1), tw1, K1);
  const cplx<T>* C = gC<T>(pm) + (size_t)z * K1 * h;
  stage2d<NT, cplx<T>>(K1, h, [&](int y, int k) { return C[y * h + k]; },
                       [&](int y, int k, cplx<T> v) { A[k * cs + y] = v; });
  cplx<T>* cols = lds_fft<T, NT>(A, B, K1, h, cs, pm.radcode[1], pm.nrad[1], tw1, T(1));
  cplx<T>* rows = cols == A ? B : A;
  for2d<NT>(K1 / 2, K0, [&](int m, int k) {
    cplx<T> X, Y;
    if (k < h) {
      X = cols[k * cs + 2 * m];
      Y = cols[k * cs + 2 * m + 1];
      if (k == 0 || 2 * k == K0) { X.y = T(0); Y.y = T(0); }
    } else {
      X = cols[(K0 - k) * cs + 2 * m];
      Y = cols[(K0 - k) * cs + 2 * m + 1];
      X.y = -X.y;
      Y.y = -Y.y;
    }
    cplx<T> v;
    v.x = X.x - Y.y;
    v.y = X.y + Y.x;
    rows[m * rs + k] = v;
  });
  cplx<T>* res = lds_fft<T, NT>(rows, cols, K0, K1 / 2, rs, pm.radcode[0], pm.nrad[0], tw0, T(1));
  T* phi = gPhi<T>(pm) + (size_t)z * K1 * K0;
  for2d<NT>(K1 / 2, K0, [&](int m, int x) {
    const cplx<T> v = res[m * rs + x];
    phi[(2 * m) * K0 + x] = v.x;
    phi[(2 * m + 1) * K0 + x] = v.y;
  });
}

// LDS bytes of the plane kernels; 0 when the planes do not fit.
static size_t plane_lds(const PmeView& pm, size_t csz) {
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh;
  const size_t bufsz =
      std::max<size_t>((size_t)(K1 / 2) * (K0 + 1), (size_t)h * (K1 + 1));
  const size_t bytes = (2 * bufsz + K0 + K1) * csz;
  return bytes <= kPlaneLdsMax ? bytes : 0;
}

// ------------------------------------------------------------ launcher
static int pick_batch(int h) {
  int best = 0;
  for (int d = 1; d <= 24; ++d)
    if (h % d == 0) best = d;
  return best >= 4 ? best : 16;
}

template <typename T>
static void z_conv(const PmeView& pm, Reduce& red, int blocks, size_t shz, int nbz, hipStream_t st,
                   bool vir) {
  red.nparts[pm.erec_slot] = blocks;
  if (vir) {
    hipLaunchKernelGGL((k_fft_z_conv<T, true>), dim3(blocks), dim3(kBlock), shz, st, pm, red, nbz);
    for (int k = 0; k < 6; ++k) red.nparts[S_VRK + k] = blocks;
  } else {
    hipLaunchKernelGGL((k_fft_z_conv<T, false>), dim3(blocks), dim3(kBlock), shz, st, pm, red, nbz);
  }
}

template <typename T>
static void convolution_t(const PmeView& pm, Reduce& red, bool mixed, hipStream_t st, bool vir) {
  const int K0 = pm.K[0], K1 = pm.K[1], K2 = pm.K[2], h = pm.kxh;
  const size_t csz = sizeof(cplx<T>);
  const int budget = 48 * 1024;
  // lines of length N per workgroup whose two buffers (stride N + 1) fit
  // the budget, at most 24
  auto lines_for = [&](int N) {
    int nl = (int)(budget / (2 * (size_t)(N + 1) * csz));
    if (nl > 24) nl = 24;
    if (nl < 1) nl = 1;
    return nl;
  };
  auto lds_for = [&](int nl, int N) { return (2 * (size_t)nl * (N + 1) + N) * csz; };
  const int nb = pick_batch(h);
  const int nbz = std::min(nb, lines_for(K2));
  const int nkbz = (h + nbz - 1) / nbz;
  const size_t shz = lds_for(nbz, K2);
  // SIBFA_FFT_PLANES=0 forces the five-pass path (used to test it on grids
  // whose planes would fit)
  const char* env = std::getenv("SIBFA_FFT_PLANES");
  const size_t lds = (env && std::atoi(env) == 0) ? 0 : plane_lds(pm, csz);
  if (lds) {
    static bool attr = false;   // raise the dynamic LDS limit once per kernel
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_fwd<T, kPlaneThreads>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlaneLdsMax);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_inv<T, kPlaneThreads>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPlaneLdsMax);
      attr = true;
    }
    launch_spread_fold(pm, mixed, st);
    hipLaunchKernelGGL((k_fft_plane_fwd<T, kPlaneThreads>), dim3(K2), dim3(kPlaneThreads), lds, st, pm);
    z_conv<T>(pm, red, K1 * nkbz, shz, nbz, st, vir);
    hipLaunchKernelGGL((k_fft_plane_inv<T, kPlaneThreads>), dim3(K2), dim3(kPlaneThreads), lds, st, pm);
    return;
  }
  launch_spread_fold(pm, mixed, st);
  const int nlx = lines_for(K0);
  const int nrows = K1 * K2;
  const size_t shx = lds_for(nlx, K0);
  hipLaunchKernelGGL(k_fft_x_r2c<T>, dim3((nrows + nlx - 1) / nlx), dim3(kBlock), shx, st, pm, nlx);
  const int nby = std::min(nb, lines_for(K1));
  const int nkby = (h + nby - 1) / nby;
  const size_t shy = lds_for(nby, K1);
  hipLaunchKernelGGL(k_fft_y<T>, dim3(K2 * nkby), dim3(kBlock), shy, st, pm, nby, T(-1));
  z_conv<T>(pm, red, K1 * nkbz, shz, nbz, st, vir);
  hipLaunchKernelGGL(k_fft_y<T>, dim3(K2 * nkby), dim3(kBlock), shy, st, pm, nby, T(1));
  hipLaunchKernelGGL(k_fft_x_c2r<T>, dim3((nrows + nlx - 1) / nlx), dim3(kBlock), shx, st, pm, nlx);
}

void launch_convolution(const PmeView& pm, Reduce& red, bool mixed, hipStream_t st, bool virial) {
  if (mixed) convolution_t<float>(pm, red, mixed, st, virial);
  else convolution_t<double>(pm, red, mixed, st, virial);
}

}  // namespace sibfa
