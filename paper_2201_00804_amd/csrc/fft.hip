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

template <typename T, int R>
__device__ __forceinline__ void stockham_stage(const cplx<T>* in, cplx<T>* out, int N, int nl,
                                               int ls, int Ns, const cplx<T>* tw, T sgn) {
  const int nb = N / R;
  const int twstep = N / (Ns * R);
  for (int bt = threadIdx.x; bt < nl * nb; bt += blockDim.x) {
    const int line = bt / nb, j = bt - line * nb;
    const cplx<T>* src = in + line * ls;
    cplx<T>* dst = out + line * ls;
    const int k = j % Ns;
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cplx<T> a = src[j + r * nb];
      if (r > 0 && Ns > 1) {
        cplx<T> w = tw[k * r * twstep];   // < N: k < Ns, r < R, twstep = N / (Ns R)
        w.y *= -sgn;   // table holds exp(-2 pi i m/N); inverse uses the conjugate
        a = cmul<T>(a, w);
      }
      v[r] = a;
    }
    dft_small<T, R>(v, sgn);
    const int o = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * Ns] = v[r];
  }
}

// Transform nl lines of length N, line stride ls, held in a (scratch b);
// returns the buffer holding the result.  Every thread of the block must
// call it.
template <typename T>
__device__ cplx<T>* lds_fft(cplx<T>* a, cplx<T>* b, int N, int nl, int ls, const int* rad,
                            int nrad, const cplx<T>* tw, T sgn) {
  int Ns = 1;
  cplx<T>* in = a;
  cplx<T>* out = b;
  for (int st = 0; st < nrad; ++st) {
    __syncthreads();
    const int R = rad[st];
    if (R == 4) stockham_stage<T, 4>(in, out, N, nl, ls, Ns, tw, sgn);
    else if (R == 2) stockham_stage<T, 2>(in, out, N, nl, ls, Ns, tw, sgn);
    else if (R == 3) stockham_stage<T, 3>(in, out, N, nl, ls, Ns, tw, sgn);
    else stockham_stage<T, 5>(in, out, N, nl, ls, Ns, tw, sgn);
    Ns *= R;
    cplx<T>* t = in; in = out; out = t;
  }
  __syncthreads();
  return in;
}

// Copies the axis' twiddle table into LDS (after the two line buffers);
// the caller's first barrier (inside lds_fft) orders it before use.
template <typename T>
__device__ __forceinline__ const cplx<T>* stage_twiddles(const cplx<T>* src, cplx<T>* dst, int N) {
  for (int k = threadIdx.x; k < N; k += blockDim.x) dst[k] = src[k];
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

// ---- x pass, real to half complex.  Block: nl rows.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_x_r2c(PmeView pm, int nl) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[0];
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nl * N;
  const int nrows = pm.K[1] * pm.K[2];
  const int row0 = blockIdx.x * nl;
  const int rows = min(nl, nrows - row0);
  const T* Q = gQ<T>(pm);
  for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
    const int l = e / N, x = e - l * N;
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (l < rows) {
      v.x = Q[(size_t)(row0 + l) * N + x];
    }
    a[e] = v;
  }
  const cplx<T>* tw = stage_twiddles<T>(gTw<T>(pm, 0), b + nl * N, N);
  cplx<T>* res = lds_fft<T>(a, b, N, nl, N, pm.rad[0], pm.nrad[0], tw, T(-1));
  cplx<T>* C = gC<T>(pm);
  const int h = pm.kxh;
  for (int e = threadIdx.x; e < nl * h; e += blockDim.x) {
    const int l = e / h, k = e - l * h;
    if (l < rows) C[(size_t)(row0 + l) * h + k] = res[l * N + k];
  }
}

// ---- y pass (both directions).  Block: (z, block of nb consecutive kx).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_y(PmeView pm, int nb, T sgn) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[1], h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nb * N;
  const int nkb = (h + nb - 1) / nb;
  const int z = blockIdx.x / nkb;
  const int kx0 = (blockIdx.x - z * nkb) * nb;
  const int cols = min(nb, h - kx0);
  cplx<T>* C = gC<T>(pm);
  for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
    const int y = e / nb, c = e - y * nb;
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (c < cols) v = C[((size_t)z * N + y) * h + kx0 + c];
    a[c * N + y] = v;
  }
  const cplx<T>* tw = stage_twiddles<T>(gTw<T>(pm, 1), b + nb * N, N);
  cplx<T>* res = lds_fft<T>(a, b, N, nb, N, pm.rad[1], pm.nrad[1], tw, sgn);
  for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
    const int y = e / nb, c = e - y * nb;
    if (c < cols) C[((size_t)z * N + y) * h + kx0 + c] = res[c * N + y];
  }
}

// ---- z pass: forward, influence function, inverse.  Block: (y, kx block).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_z_conv(PmeView pm, Reduce red, int nb) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[2], K1 = pm.K[1], h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nb * N;
  const int nkb = (h + nb - 1) / nb;
  const int y = blockIdx.x / nkb;
  const int kx0 = (blockIdx.x - y * nkb) * nb;
  const int cols = min(nb, h - kx0);
  cplx<T>* C = gC<T>(pm);
  for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
    const int z = e / nb, c = e - z * nb;
    cplx<T> v;
    v.x = T(0); v.y = T(0);
    if (c < cols) v = C[((size_t)z * K1 + y) * h + kx0 + c];
    a[c * N + z] = v;
  }
  const cplx<T>* tw = stage_twiddles<T>(gTw<T>(pm, 2), b + nb * N, N);
  cplx<T>* res = lds_fft<T>(a, b, N, nb, N, pm.rad[2], pm.nrad[2], tw, T(-1));
  const T* G = gG<T>(pm);
  double e_part = 0.0;
  for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
    const int c = e / N, z = e - c * N;
    if (c < cols) {
      const int kx = kx0 + c;
      const T g = G[((size_t)z * K1 + y) * h + kx];
      cplx<T> v = res[e];
      const double mult = (kx == 0 || 2 * kx == pm.K[0]) ? 1.0 : 2.0;
      e_part += 0.5 * mult * (double)g * ((double)v.x * v.x + (double)v.y * v.y);
      v.x *= g; v.y *= g;
      res[e] = v;
    }
  }
  cplx<T>* other = (res == a) ? b : a;
  cplx<T>* res2 = lds_fft<T>(res, other, N, nb, N, pm.rad[2], pm.nrad[2], tw, T(1));
  for (int e = threadIdx.x; e < nb * N; e += blockDim.x) {
    const int z = e / nb, c = e - z * nb;
    if (c < cols) C[((size_t)z * K1 + y) * h + kx0 + c] = res2[c * N + z];
  }
  block_partial(e_part, red, pm.erec_slot);
}

// ---- x pass, half complex to real.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft_x_c2r(PmeView pm, int nl) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int N = pm.K[0], h = pm.kxh;
  cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* b = a + nl * N;
  const int nrows = pm.K[1] * pm.K[2];
  const int row0 = blockIdx.x * nl;
  const int rows = min(nl, nrows - row0);
  const cplx<T>* C = gC<T>(pm);
  for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
    const int l = e / N, k = e - l * N;
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
    a[e] = v;
  }
  const cplx<T>* tw = stage_twiddles<T>(gTw<T>(pm, 0), b + nl * N, N);
  cplx<T>* res = lds_fft<T>(a, b, N, nl, N, pm.rad[0], pm.nrad[0], tw, T(1));
  T* phi = gPhi<T>(pm);
  for (int e = threadIdx.x; e < nl * N; e += blockDim.x) {
    const int l = e / N, x = e - l * N;
    if (l < rows) phi[(size_t)(row0 + l) * N + x] = res[e].x;
  }
}

// ---- whole z-planes in LDS (grids whose planes fit in a workgroup's LDS)
// Forward: transform pairs of real rows of Q (folded from the spreading
// tiles by k_spread_fold) as one complex line (rows y and y + 1 as real and imaginary
// parts), split them into the two half spectra, then transform the columns
// (one per kx) along y; writes C[z][y][kx].
// Inverse: columns along y, then pairs of Hermitian-completed rows combined
// as X + iY into one complex line, inverse, real and imaginary parts ->
// rows y and y + 1 of phi.  The imaginary parts of the kx = 0 and kx = K0/2
// entries are dropped, as a real inverse does.
constexpr int kPlaneThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kPlaneThreads) void k_fft_plane_fwd(PmeView pm) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh, z = blockIdx.x;
  const int cs = K1 + 1;                        // column stride (odd: no bank conflicts)
  const int bufsz = max((K1 / 2) * K0, h * cs);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + bufsz;
  cplx<T>* tw0 = B + bufsz;
  cplx<T>* tw1 = tw0 + K0;
  stage_twiddles<T>(gTw<T>(pm, 0), tw0, K0);
  stage_twiddles<T>(gTw<T>(pm, 1), tw1, K1);
  const T* Q = gQ<T>(pm) + (size_t)z * K1 * K0;
  for (int e = threadIdx.x; e < (K1 / 2) * K0; e += blockDim.x) {
    const int m = e / K0, x = e - m * K0;
    cplx<T> v;
    v.x = Q[(2 * m) * K0 + x];
    v.y = Q[(2 * m + 1) * K0 + x];
    A[e] = v;
  }
  cplx<T>* rows = lds_fft<T>(A, B, K0, K1 / 2, K0, pm.rad[0], pm.nrad[0], tw0, T(-1));
  cplx<T>* cols = rows == A ? B : A;
  for (int e = threadIdx.x; e < (K1 / 2) * h; e += blockDim.x) {
    const int m = e / h, k = e - m * h;
    const cplx<T> zk = rows[m * K0 + k];
    const cplx<T> zn = rows[m * K0 + (k == 0 ? 0 : K0 - k)];
    cplx<T> X, Y;
    X.x = T(0.5) * (zk.x + zn.x);
    X.y = T(0.5) * (zk.y - zn.y);
    Y.x = T(0.5) * (zk.y + zn.y);
    Y.y = T(0.5) * (zn.x - zk.x);
    cols[k * cs + 2 * m] = X;
    cols[k * cs + 2 * m + 1] = Y;
  }
  cplx<T>* res = lds_fft<T>(cols, rows, K1, h, cs, pm.rad[1], pm.nrad[1], tw1, T(-1));
  cplx<T>* C = gC<T>(pm);
  for (int e = threadIdx.x; e < K1 * h; e += blockDim.x) {
    const int y = e / h, k = e - y * h;
    C[((size_t)z * K1 + y) * h + k] = res[k * cs + y];
  }
}

template <typename T>
__global__ __launch_bounds__(kPlaneThreads) void k_fft_plane_inv(PmeView pm) {
  if (stopped(pm.stop)) return;
  extern __shared__ char smem[];
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh, z = blockIdx.x;
  const int cs = K1 + 1;
  const int bufsz = max((K1 / 2) * K0, h * cs);
  cplx<T>* A = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* B = A + bufsz;
  cplx<T>* tw0 = B + bufsz;
  cplx<T>* tw1 = tw0 + K0;
  stage_twiddles<T>(gTw<T>(pm, 0), tw0, K0);
  stage_twiddles<T>(gTw<T>(pm, 1), tw1, K1);
  const cplx<T>* C = gC<T>(pm);
  for (int e = threadIdx.x; e < K1 * h; e += blockDim.x) {
    const int y = e / h, k = e - y * h;
    A[k * cs + y] = C[((size_t)z * K1 + y) * h + k];
  }
  cplx<T>* cols = lds_fft<T>(A, B, K1, h, cs, pm.rad[1], pm.nrad[1], tw1, T(1));
  cplx<T>* rows = cols == A ? B : A;
  for (int e = threadIdx.x; e < (K1 / 2) * K0; e += blockDim.x) {
    const int m = e / K0, k = e - m * K0;
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
    rows[m * K0 + k] = v;
  }
  cplx<T>* res = lds_fft<T>(rows, cols, K0, K1 / 2, K0, pm.rad[0], pm.nrad[0], tw0, T(1));
  T* phi = gPhi<T>(pm);
  for (int e = threadIdx.x; e < (K1 / 2) * K0; e += blockDim.x) {
    const int m = e / K0, x = e - m * K0;
    const cplx<T> v = res[e];
    phi[((size_t)z * K1 + 2 * m) * K0 + x] = v.x;
    phi[((size_t)z * K1 + 2 * m + 1) * K0 + x] = v.y;
  }
}

// LDS bytes of the plane kernels; 0 when the planes do not fit.
static size_t plane_lds(const PmeView& pm, size_t csz) {
  const int K0 = pm.K[0], K1 = pm.K[1], h = pm.kxh;
  const size_t bufsz = std::max<size_t>((size_t)(K1 / 2) * K0, (size_t)h * (K1 + 1));
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
static void convolution_t(const PmeView& pm, Reduce& red, bool mixed, hipStream_t st) {
  const int K0 = pm.K[0], K1 = pm.K[1], K2 = pm.K[2], h = pm.kxh;
  const size_t csz = sizeof(cplx<T>);
  // SIBFA_FFT_PLANES=0 forces the five-pass path (used to test it on grids
  // whose planes would fit)
  const char* env = std::getenv("SIBFA_FFT_PLANES");
  const size_t lds = (env && std::atoi(env) == 0) ? 0 : plane_lds(pm, csz);
  if (lds) {
    static bool attr = false;   // raise the dynamic LDS limit once per kernel
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_fwd<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_plane_inv<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr = true;
    }
    const int nb = pick_batch(h);
    const int budget = 48 * 1024;
    int nbz = (int)(budget / (2 * K2 * csz));
    nbz = std::max(1, std::min(nbz, std::min(nb, 24)));
    const int nkbz = (h + nbz - 1) / nbz;
    const size_t shz = (2 * (size_t)nbz + 1) * K2 * csz;
    launch_spread_fold(pm, mixed, st);
    hipLaunchKernelGGL(k_fft_plane_fwd<T>, dim3(K2), dim3(kPlaneThreads), lds, st, pm);
    red.nparts[pm.erec_slot] = K1 * nkbz;
    hipLaunchKernelGGL(k_fft_z_conv<T>, dim3(K1 * nkbz), dim3(kBlock), shz, st, pm, red, nbz);
    hipLaunchKernelGGL(k_fft_plane_inv<T>, dim3(K2), dim3(kPlaneThreads), lds, st, pm);
    return;
  }
  launch_spread_fold(pm, mixed, st);
  const int budget = 48 * 1024;
  auto lines_for = [&](int N) {
    int nl = (int)(budget / (2 * N * csz));
    if (nl > 24) nl = 24;
    if (nl < 1) nl = 1;
    return nl;
  };
  const int nlx = lines_for(K0);
  const int nrows = K1 * K2;
  const size_t shx = (2 * (size_t)nlx + 1) * K0 * csz;
  hipLaunchKernelGGL(k_fft_x_r2c<T>, dim3((nrows + nlx - 1) / nlx), dim3(kBlock), shx, st, pm, nlx);
  const int nb = pick_batch(h);
  const int nby = nb < lines_for(K1) ? nb : lines_for(K1);
  const int nkby = (h + nby - 1) / nby;
  const size_t shy = (2 * (size_t)nby + 1) * K1 * csz;
  hipLaunchKernelGGL(k_fft_y<T>, dim3(K2 * nkby), dim3(kBlock), shy, st, pm, nby, T(-1));
  const int nbz = nb < lines_for(K2) ? nb : lines_for(K2);
  const int nkbz = (h + nbz - 1) / nbz;
  const size_t shz = (2 * (size_t)nbz + 1) * K2 * csz;
  red.nparts[pm.erec_slot] = K1 * nkbz;
  hipLaunchKernelGGL(k_fft_z_conv<T>, dim3(K1 * nkbz), dim3(kBlock), shz, st, pm, red, nbz);
  hipLaunchKernelGGL(k_fft_y<T>, dim3(K2 * nkby), dim3(kBlock), shy, st, pm, nby, T(1));
  hipLaunchKernelGGL(k_fft_x_c2r<T>, dim3((nrows + nlx - 1) / nlx), dim3(kBlock), shx, st, pm, nlx);
}

void launch_convolution(const PmeView& pm, Reduce& red, bool mixed, hipStream_t st) {
  if (mixed) convolution_t<float>(pm, red, mixed, st);
  else convolution_t<double>(pm, red, mixed, st);
}

}  // namespace sibfa
