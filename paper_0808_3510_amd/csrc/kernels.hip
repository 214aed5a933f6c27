// CDNA4 (gfx950) kernels of the NUFFT-based planar photoacoustic
// reconstruction.  Every kernel runs 256-thread workgroups over a list of work
// items (instance, tile or line); items come either one per workgroup or from
// a device work counter drained by a persistent grid (batched form).
//
// Stages (see pat.h for the operators they compose):
//   k_tr_x1_r2c   DFT over the first detector axis, real input, half spectrum
//   k_tr_x2       DFT over the second detector axis (either direction)
//   k_tr_c2r_k1   inverse DFT over the first axis from the half spectrum, real part
//   k_line_fft    DFT along contiguous lines (depth axis)
//   k_line_a2     deconvolve by 1/Psi, centre, zero-pad to c*nt, FFT (eq. nufft-c)
//   k_line_a2t    its transpose: inverse FFT, pick, multiply by 1/Psi
//   k_line_interp type-2 interpolation with 2cK Kaiser-Bessel taps (eq. nufft-a)
//                 and the Jacobian weight (eq. fft-0)
//   k_line_spread its transpose (type-1), gathered per grid cell over the
//                 monotone node list of the line: no atomics, deterministic
//
// All uniform FFTs are in-place decimation-in-frequency mixed-radix transforms
// in LDS; bin k ends at position perm[k] (a table built by the host plan).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.h"
#include "pat_internal.h"

namespace pat {

// ---------------------------------------------------------------------------
// complex helpers

template <typename T>
struct cx {
  T x, y;
};
struct bf2 {
  uint16_t x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cx<T> cscl(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> cmi(cx<T> a) { return mk(a.y, -a.x); }

__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ void m_sincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void m_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }

// Storage of the oversampled grid: the compute type itself, or bf16 pairs.
template <typename T, typename G>
struct GridIO;
template <typename T>
struct GridIO<T, cx<T>> {
  static __device__ __forceinline__ cx<T> ld(const cx<T>* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ void st(cx<T>* p, size_t i, cx<T> v) { p[i] = v; }
};
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even (finite values)
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
template <>
struct GridIO<float, bf2> {
  static __device__ __forceinline__ cx<float> ld(const bf2* p, size_t i) {
    bf2 v = p[i];
    return mk(bf2f(v.x), bf2f(v.y));
  }
  static __device__ __forceinline__ void st(bf2* p, size_t i, cx<float> v) {
    bf2 o;
    o.x = f2bf(v.x);
    o.y = f2bf(v.y);
    p[i] = o;
  }
};

// ---------------------------------------------------------------------------
// LDS FFT: forward DFT  X[k] = sum_n x[n] exp(-2 pi i n k / L), in place,
// decimation in frequency.  Stage s with radix R works on sub-transforms of
// length Li (L, L/R_1, ...): butterfly j of a block reads x[j + r*Li/R],
// forms the R-point DFT, multiplies output d by exp(-2 pi i j d / Li) and
// writes it back to position j + d*Li/R.  Transform b's element e lives at
// buf[b*bs + e*es]; threads are mapped batch-fastest.

template <typename T, int R>
__device__ __forceinline__ void dft_small(cx<T>* v, const cx<T>* __restrict__ tw, int L) {
  if constexpr (R == 2) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cx<T> s13 = cadd(v[1], v[3]), d13 = cmi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else if constexpr (R == 8) {
    const T h = T(0.70710678118654752440084436210484904);
    // even / odd 4-point DFTs
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<T, 4>(e, tw, L);
    dft_small<T, 4>(o, tw, L);
    // o[d] *= exp(-2 pi i d / 8)
    cx<T> o1 = mk(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    cx<T> o2 = cmi(o[2]);
    cx<T> o3 = mk(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  } else {
    // odd prime: direct R-point DFT with roots from the L-point table
    const int step = L / R;
    cx<T> w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) w[q] = tw[q * step];
    cx<T> y[R];
#pragma unroll
    for (int d = 0; d < R; ++d) {
      cx<T> acc = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) acc = cadd(acc, cmul(v[r], w[(r * d) % R]));
      y[d] = acc;
    }
#pragma unroll
    for (int d = 0; d < R; ++d) v[d] = y[d];
  }
}

template <typename T, int R>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int Li, int L, const cx<T>* __restrict__ tw,
                                          int nb, int bs, int es) {
  const int sub = Li / R;
  const int tws = L / Li;
  const int total = (L / R) * nb;
  for (int id = threadIdx.x; id < total; id += kBlock) {
    const int bf = id / nb;
    const int b = id - bf * nb;
    const int blk = bf / sub;
    const int j = bf - blk * sub;
    cx<T>* p = buf + b * bs + (blk * Li + j) * es;
    const int st = sub * es;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = p[r * st];
    dft_small<T, R>(v, tw, L);
#pragma unroll
    for (int d = 1; d < R; ++d) v[d] = cmul(v[d], tw[j * d * tws]);
#pragma unroll
    for (int r = 0; r < R; ++r) p[r * st] = v[r];
  }
}

template <typename T>
__device__ void fft_lds(cx<T>* buf, const FftDesc& d, const cx<T>* __restrict__ tw_all, int nb, int bs,
                        int es) {
  const cx<T>* tw = tw_all + d.tw;
  const int L = d.L;
  int Li = L;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.rad[s];
    switch (R) {
      case 2: fft_stage<T, 2>(buf, Li, L, tw, nb, bs, es); break;
      case 3: fft_stage<T, 3>(buf, Li, L, tw, nb, bs, es); break;
      case 4: fft_stage<T, 4>(buf, Li, L, tw, nb, bs, es); break;
      case 5: fft_stage<T, 5>(buf, Li, L, tw, nb, bs, es); break;
      case 7: fft_stage<T, 7>(buf, Li, L, tw, nb, bs, es); break;
      case 8: fft_stage<T, 8>(buf, Li, L, tw, nb, bs, es); break;
      case 11: fft_stage<T, 11>(buf, Li, L, tw, nb, bs, es); break;
      case 13: fft_stage<T, 13>(buf, Li, L, tw, nb, bs, es); break;
      case 17: fft_stage<T, 17>(buf, Li, L, tw, nb, bs, es); break;
      case 19: fft_stage<T, 19>(buf, Li, L, tw, nb, bs, es); break;
      case 23: fft_stage<T, 23>(buf, Li, L, tw, nb, bs, es); break;
      default: break;  // the host plan only emits the radices above
    }
    __syncthreads();
    Li /= R;
  }
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel interpolation kernel.  With s = sqrt(K^2 - u^2), |u| <= K,
//   Psi_hat(u) I0(alpha K) / (2 e^{alpha K}) = e^{alpha (s - K)} (1 - e^{-2 alpha s}) / (2 s)
// (the transform of Section 3.2 with the large factor e^{alpha K} / I0(alpha K)
// moved into the deconvolution table), limit alpha e^{-alpha K} at s -> 0.

template <typename T>
__device__ __forceinline__ T kb_phi(T u, T K, T alpha) {
  T s2 = (K - u) * (K + u);
  s2 = s2 > T(0) ? s2 : T(0);
  const T s = m_sqrt(s2);
  const T as = alpha * s;
  T v;
  if (as > T(1e-3)) {
    v = -m_expm1(T(-2) * as) / (T(2) * s);
  } else {
    v = alpha * (T(1) - as + T(2) / T(3) * as * as);
  }
  return m_exp(alpha * (s - K)) * v;
}

// Node position on the oversampled grid: x = c nu, first tap j0 = floor(x - cK) + 1,
// fractional offset delta = x - j0 in (cK - 1, cK].  Formed in double.
struct NodePos {
  int j0;
  double delta;
};
__device__ __forceinline__ NodePos node_pos(double nu, double c, double ck) {
  const double x = c * nu;
  NodePos p;
  p.j0 = (int)floor(x - ck) + 1;
  p.delta = x - (double)p.j0;
  return p;
}

// exp(-i pi nu), argument reduced in double to [-1, 1].
template <typename T>
__device__ __forceinline__ cx<T> phase_mpi(double nu) {
  const double r = nu - 2.0 * rint(0.5 * nu);
  T s, c;
  m_sincospi((T)r, &s, &c);
  return mk(c, -s);
}

// sum_t phi((delta - t)/c) U[(j0 + t) mod m] times exp(-i pi nu)
template <typename T>
__device__ __forceinline__ cx<T> interp_eval(const cx<T>* U, int m, int taps, double nu, const Inst& I,
                                             T cinv, T K, T alpha) {
  const NodePos np = node_pos(nu, I.c, I.ck);
  const T delta = (T)np.delta;
  int jm = np.j0 % m;
  if (jm < 0) jm += m;
  cx<T> acc = mk(T(0), T(0));
  for (int t = 0; t < taps; ++t) {
    const T w = kb_phi<T>((delta - T(t)) * cinv, K, alpha);
    const cx<T> g = U[jm];
    acc.x += w * g.x;
    acc.y += w * g.y;
    ++jm;
    if (jm == m) jm = 0;
  }
  return cmul(acc, phase_mpi<T>(nu));
}

// ---------------------------------------------------------------------------
// Work distribution

struct StageArgs {
  int32_t n;      // instances
  int32_t total;  // work items over all instances
  int32_t off[kMaxBatch + 1];
  const Inst* inst[kMaxBatch];
  const void* in[kMaxBatch];
  void* out[kMaxBatch];
  uint32_t* counter;  // persistent queue, or nullptr: item = blockIdx.x
  int32_t len_nz;     // transverse passes: lines have nz (else nt) samples
  int32_t mode;       // FFT direction (0 forward, 1 inverse) / interp, spread mode
};

__device__ __forceinline__ int next_item(const StageArgs& a, int iter, int* s_item) {
  int item;
  if (a.counter) {
    __syncthreads();
    if (threadIdx.x == 0) *s_item = (int)atomicAdd(a.counter, 1u);
    __syncthreads();
    item = *s_item;
  } else {
    item = iter == 0 ? (int)blockIdx.x : a.total;
  }
  return __builtin_amdgcn_readfirstlane(item);
}

__device__ __forceinline__ int find_inst(const StageArgs& a, int item) {
  int i = 0;
  while (i + 1 < a.n && a.off[i + 1] <= item) ++i;
  return i;
}

#define PAT_FOR_EACH_ITEM(a)                                              \
  __shared__ int s_item_;                                                 \
  for (int iter_ = 0;; ++iter_) {                                         \
    const int item_ = next_item(a, iter_, &s_item_);                      \
    if (item_ >= (a).total) break;                                        \
    const int inst_ = __builtin_amdgcn_readfirstlane(find_inst(a, item_)); \
    const Inst& I = *(a).inst[inst_];                                     \
    const int li = item_ - (a).off[inst_];

#define PAT_END_ITEM \
  __syncthreads();   \
  }

extern __shared__ __align__(16) unsigned char pat_smem[];

// ---------------------------------------------------------------------------
// Transverse passes.  Tiles of tb consecutive samples (t or z, the contiguous
// axis) by the full transform length; lane -> sample, so global accesses are
// contiguous runs of tb elements.

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tr_x1_r2c(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = I.tb;
  const int ntile = (len + tb - 1) / tb;
  const int x2 = li / ntile;
  const int t0 = (li - x2 * ntile) * tb;
  const T* in = static_cast<const T*>(a.in[inst_]);
  cx<T>* out = static_cast<cx<T>*>(a.out[inst_]);
  const int L = I.n1;
  for (int e = threadIdx.x; e < L * tb; e += kBlock) {
    const int x = e / tb;
    const int t = t0 + (e - x * tb);
    const T v = t < len ? in[((size_t)x * I.n2 + x2) * len + t] : T(0);
    buf[e] = mk(v, T(0));
  }
  __syncthreads();
  fft_lds<T>(buf, I.f1, static_cast<const cx<T>*>(I.tw), tb, 1, tb);
  const int32_t* perm = I.perm + I.f1.perm;
  for (int e = threadIdx.x; e < I.h1 * tb; e += kBlock) {
    const int k = e / tb;
    const int b = e - k * tb;
    const int t = t0 + b;
    if (t < len) out[((size_t)k * I.n2 + x2) * len + t] = buf[perm[k] * tb + b];
  }
  PAT_END_ITEM
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tr_x2(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = I.tb;
  const int ntile = (len + tb - 1) / tb;
  const int k1 = li / ntile;
  const int t0 = (li - k1 * ntile) * tb;
  cx<T>* io = static_cast<cx<T>*>(a.out[inst_]);
  const int L = I.n2;
  const bool inv = a.mode != 0;
  for (int e = threadIdx.x; e < L * tb; e += kBlock) {
    const int x = e / tb;
    const int t = t0 + (e - x * tb);
    cx<T> v = t < len ? io[((size_t)k1 * L + x) * len + t] : mk(T(0), T(0));
    buf[e] = inv ? cconj(v) : v;
  }
  __syncthreads();
  fft_lds<T>(buf, I.f2, static_cast<const cx<T>*>(I.tw), tb, 1, tb);
  const int32_t* perm = I.perm + I.f2.perm;
  for (int e = threadIdx.x; e < L * tb; e += kBlock) {
    const int k = e / tb;
    const int b = e - k * tb;
    const int t = t0 + b;
    if (t < len) {
      const cx<T> v = buf[perm[k] * tb + b];
      io[((size_t)k1 * L + k) * len + t] = inv ? cconj(v) : v;
    }
  }
  PAT_END_ITEM
}

// Inverse DFT over the first axis from bins 0..n1/2 (the others are the
// complex conjugates of their mirror bins), keeping the real part.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tr_c2r_k1(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = I.tb;
  const int ntile = (len + tb - 1) / tb;
  const int x2 = li / ntile;
  const int t0 = (li - x2 * ntile) * tb;
  const cx<T>* in = static_cast<const cx<T>*>(a.in[inst_]);
  T* out = static_cast<T*>(a.out[inst_]);
  const int L = I.n1;
  const int half = L / 2;
  for (int e = threadIdx.x; e < L * tb; e += kBlock) {
    const int k = e / tb;
    const int t = t0 + (e - k * tb);
    const int src = k <= half ? k : L - k;
    cx<T> v = t < len ? in[((size_t)src * I.n2 + x2) * len + t] : mk(T(0), T(0));
    // inverse transform as conj(FFT(conj(.))); mirrored bins are conjugated once more
    buf[e] = k <= half ? cconj(v) : v;
  }
  __syncthreads();
  fft_lds<T>(buf, I.f1, static_cast<const cx<T>*>(I.tw), tb, 1, tb);
  const int32_t* perm = I.perm + I.f1.perm;
  for (int e = threadIdx.x; e < L * tb; e += kBlock) {
    const int x = e / tb;
    const int b = e - x * tb;
    const int t = t0 + b;
    if (t < len) out[((size_t)x * I.n2 + x2) * len + t] = buf[perm[x] * tb + b].x;
  }
  PAT_END_ITEM
}

// ---------------------------------------------------------------------------
// Line stages: one frequency line (k1, k2) per work item.

__device__ __forceinline__ void line_freqs(const Inst& I, int line, double* Ak) {
  const int k1 = line / I.n2;
  const int k2i = line - k1 * I.n2;
  const int k2 = 2 * k2i < I.n2 ? k2i : k2i - I.n2;
  *Ak = I.a1 * (double)k1 * (double)k1 + I.a2 * (double)k2 * (double)k2;
}

// DFT of length nz along each line, in place.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_line_fft(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int L = I.nz;
  cx<T>* io = static_cast<cx<T>*>(a.out[inst_]) + (size_t)li * L;
  const bool inv = a.mode != 0;
  for (int j = threadIdx.x; j < L; j += kBlock) {
    const cx<T> v = io[j];
    buf[j] = inv ? cconj(v) : v;
  }
  __syncthreads();
  fft_lds<T>(buf, I.fz, static_cast<const cx<T>*>(I.tw), 1, 0, 1);
  const int32_t* perm = I.perm + I.fz.perm;
  for (int j = threadIdx.x; j < L; j += kBlock) {
    const cx<T> v = buf[perm[j]];
    io[j] = inv ? cconj(v) : v;
  }
  PAT_END_ITEM
}

// a2: u_n = G_n s_n placed at (n - nt/2) mod m, zeros elsewhere, FFT of length m.
// The centring turns the per-tap factor exp(i pi j / c) of eq. (nufft-a) into
// a shift, leaving only exp(-i pi nu) per node.
template <typename T, typename G>
__global__ __launch_bounds__(kBlock) void k_line_a2(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nt = I.nt;
  const cx<T>* g = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)li * nt;
  G* grid = static_cast<G*>(a.out[inst_]);
  const T* sn = static_cast<const T*>(I.sn);
  for (int j = threadIdx.x; j < m; j += kBlock) {
    int n = j + nt / 2;
    if (n >= m) n -= m;
    buf[j] = n < nt ? cscl(g[n], sn[n]) : mk(T(0), T(0));
  }
  __syncthreads();
  fft_lds<T>(buf, I.fm, static_cast<const cx<T>*>(I.tw), 1, 0, 1);
  const int32_t* perm = I.perm + I.fm.perm;
  for (int j = threadIdx.x; j < m; j += kBlock) GridIO<T, G>::st(grid, (size_t)li * m + j, buf[perm[j]]);
  PAT_END_ITEM
}

// transpose of a2: X_n = s_n (inverse DFT of the grid line)[(n - nt/2) mod m]
template <typename T, typename G>
__global__ __launch_bounds__(kBlock) void k_line_a2t(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nt = I.nt;
  const G* grid = static_cast<const G*>(a.in[inst_]);
  cx<T>* x = static_cast<cx<T>*>(a.out[inst_]) + (size_t)li * nt;
  const T* sn = static_cast<const T*>(I.sn);
  for (int j = threadIdx.x; j < m; j += kBlock) buf[j] = cconj(GridIO<T, G>::ld(grid, (size_t)li * m + j));
  __syncthreads();
  fft_lds<T>(buf, I.fm, static_cast<const cx<T>*>(I.tw), 1, 0, 1);
  const int32_t* perm = I.perm + I.fm.perm;
  for (int n = threadIdx.x; n < nt; n += kBlock) {
    int pos = n - nt / 2;
    if (pos < 0) pos += m;
    x[n] = cscl(cconj(buf[perm[pos]]), sn[n]);
  }
  PAT_END_ITEM
}

// a3: type-2 interpolation.  mode 0 (R): node sign(l) nu+, weight
// wcoef |l| / nu+ (0 at l = 0), mean of the nodes -+nu+ on l = -nz/2.
// mode 1 (A^T): mean of the nodes +-nu+ for every l, no weight.
template <typename T, typename G>
__global__ __launch_bounds__(kBlock) void k_line_interp(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nz = I.nz;
  const G* grid = static_cast<const G*>(a.in[inst_]);
  cx<T>* out = static_cast<cx<T>*>(a.out[inst_]) + (size_t)li * nz;
  for (int j = threadIdx.x; j < m; j += kBlock) buf[j] = GridIO<T, G>::ld(grid, (size_t)li * m + j);
  __syncthreads();
  double Ak;
  line_freqs(I, li, &Ak);
  const T cinv = T(1.0 / I.c), K = T(I.K), alpha = T(I.alpha);
  for (int il = threadIdx.x; il < nz; il += kBlock) {
    const int l = 2 * il < nz ? il : il - nz;
    const double nup = sqrt(Ak + I.b * (double)l * (double)l);
    cx<T> v;
    if (a.mode == 0) {
      if (l == 0) {
        v = mk(T(0), T(0));
      } else {
        const double w = I.wcoef * (double)(l < 0 ? -l : l) / nup * I.scale;
        if (2 * l == -nz) {
          v = cadd(interp_eval<T>(buf, m, I.taps, -nup, I, cinv, K, alpha),
                   interp_eval<T>(buf, m, I.taps, nup, I, cinv, K, alpha));
          v = cscl(v, T(0.5 * w));
        } else {
          v = cscl(interp_eval<T>(buf, m, I.taps, l > 0 ? nup : -nup, I, cinv, K, alpha), T(w));
        }
      }
    } else {
      v = cadd(interp_eval<T>(buf, m, I.taps, nup, I, cinv, K, alpha),
               interp_eval<T>(buf, m, I.taps, -nup, I, cinv, K, alpha));
      v = cscl(v, T(0.5 * I.scale));
    }
    out[il] = v;
  }
  PAT_END_ITEM
}

// first index i in [0, n) with key[i] >= v (n if none)
__device__ __forceinline__ int lower_bound_i(const int* key, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (key[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// a6: type-1 spreading, the transpose of k_line_interp's sum.  The line's
// nodes are listed in increasing order (they are monotone in l by
// construction), each with its first tap j0 and value; every grid cell then
// gathers the nodes whose 2cK-tap window covers it (binary search on j0),
// for each periodic image of the cell.
//   mode 0 (R^T): nodes sign(l) nu+ for l = -nz/2 .. nz/2-1 plus +nu+(nz/2);
//     value conj(W exp(-i pi nu) scale) Qhat_l, halved on the Nyquist plane,
//     whose value feeds both -nu+ and +nu+.
//   mode 1 (A): nodes -nu+(nz/2) .. -nu+(0), +nu+(0) .. +nu+(nz/2); value
//     (scale / 2) exp(i pi nu) (F_l + F_-l) (single term at l = 0, -nz/2).
template <typename T, typename G>
__global__ __launch_bounds__(kBlock) void k_line_spread(StageArgs a) {
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nz = I.nz, taps = I.taps;
  const int nn = a.mode == 0 ? nz + 1 : nz + 2;
  cx<T>* val = reinterpret_cast<cx<T>*>(pat_smem);
  T* dl = reinterpret_cast<T*>(val + nn);
  int* j0s = reinterpret_cast<int*>(dl + nn);
  const cx<T>* F = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)li * nz;
  G* grid = static_cast<G*>(a.out[inst_]);
  double Ak;
  line_freqs(I, li, &Ak);
  const int half = nz / 2;
  for (int i = threadIdx.x; i < nn; i += kBlock) {
    double nu, coef;
    cx<T> q;
    if (a.mode == 0) {
      const int l = i < nz ? i - half : half;
      const double nup = sqrt(Ak + I.b * (double)l * (double)l);
      const int lm = l < 0 ? l + nz : (l == half ? half : l);
      q = F[lm];
      if (i == nz) {
        nu = nup;
        coef = 0.5 * I.wcoef * (double)half / nup;
      } else {
        nu = l > 0 ? nup : (l < 0 ? -nup : 0.0);
        coef = l == 0 ? 0.0 : I.wcoef * (double)(l < 0 ? -l : l) / nup;
        if (l == -half) coef *= 0.5;
      }
      coef *= I.scale;
    } else {
      int mp;
      double sg;
      if (i <= half) {
        mp = half - i;
        sg = -1.0;
      } else {
        mp = i - half - 1;
        sg = 1.0;
      }
      const double nup = sqrt(Ak + I.b * (double)mp * (double)mp);
      nu = sg * nup;
      q = F[mp];
      if (mp != 0 && mp != half) q = cadd(q, F[nz - mp]);
      coef = 0.5 * I.scale;
    }
    const NodePos np = node_pos(nu, I.c, I.ck);
    val[i] = cscl(cmul(q, cconj(phase_mpi<T>(nu))), T(coef));
    dl[i] = (T)np.delta;
    j0s[i] = np.j0;
  }
  __syncthreads();
  const T cinv = T(1.0 / I.c), K = T(I.K), alpha = T(I.alpha);
  const int jlo = j0s[0];
  const int jhi = j0s[nn - 1] + taps - 1;
  for (int j = threadIdx.x; j < m; j += kBlock) {
    cx<T> acc = mk(T(0), T(0));
    // first periodic image j + q m that can be covered
    int q0 = jlo - j;
    q0 = q0 >= 0 ? (q0 + m - 1) / m : -((-q0) / m);
    for (int jp = j + q0 * m; jp <= jhi; jp += m) {
      const int lo = lower_bound_i(j0s, nn, jp - taps + 1);
      const int hi = lower_bound_i(j0s, nn, jp + 1);
      for (int i = lo; i < hi; ++i) {
        const T w = kb_phi<T>((dl[i] - T(jp - j0s[i])) * cinv, K, alpha);
        acc.x += w * val[i].x;
        acc.y += w * val[i].y;
      }
    }
    GridIO<T, G>::st(grid, (size_t)li * m + j, acc);
  }
  PAT_END_ITEM
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host launchers

namespace {

int g_num_cu = 0;

int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  return g_num_cu;
}

template <typename K>
hipError_t launch(K kernel, const char* name, StageArgs& a, size_t shmem, hipStream_t st, StageTimer* tm) {
  if (a.total <= 0) return hipSuccess;
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  int grid = a.total;
  if (a.counter) {
    const int cap = 8 * num_cu();
    grid = a.total < cap ? a.total : cap;
  }
  if (tm) tm->begin(name, st);
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), shmem, st, a);
  hipError_t e = hipGetLastError();
  if (tm) tm->end(st);
  return e;
}

enum Items { IT_X1, IT_X2, IT_LINES, IT_C2R };

int items_of(const Inst& I, Items kind, bool nz) {
  const int len = nz ? I.nz : I.nt;
  const int ntile = (len + I.tb - 1) / I.tb;
  switch (kind) {
    case IT_X1: return I.n2 * ntile;
    case IT_X2: return I.n2 > 1 ? I.h1 * ntile : 0;
    case IT_LINES: return I.lines;
    case IT_C2R: return I.n2 * ntile;
  }
  return 0;
}

template <typename T, typename G>
struct Runner {
  int n;
  const Inst* h;
  const Inst* const* d;
  uint32_t* counters;
  int next_counter = 0;
  hipStream_t st;
  StageTimer* tm;

  static constexpr size_t cs = sizeof(cx<T>);

  // in/out pointer of instance i for a stage, from a selector
  StageArgs base(Items kind, bool nz, int mode) {
    StageArgs a;
    a.n = n;
    a.len_nz = nz ? 1 : 0;
    a.mode = mode;
    a.off[0] = 0;
    for (int i = 0; i < n; ++i) {
      a.inst[i] = d[i];
      a.off[i + 1] = a.off[i] + items_of(h[i], kind, nz);
    }
    a.total = a.off[n];
    a.counter = counters ? counters + (next_counter++ % kNumCounters) : nullptr;
    return a;
  }

  size_t max_over(size_t (*f)(const Inst&)) const {
    size_t m = 0;
    for (int i = 0; i < n; ++i) {
      const size_t v = f(h[i]);
      if (v > m) m = v;
    }
    return m;
  }

  static size_t sh_x1(const Inst& I) { return (size_t)I.n1 * I.tb * cs; }
  static size_t sh_x2(const Inst& I) { return (size_t)I.n2 * I.tb * cs; }
  static size_t sh_z(const Inst& I) { return (size_t)I.nz * cs; }
  static size_t sh_m(const Inst& I) { return (size_t)I.m * cs; }
  static size_t sh_spread(const Inst& I) { return (size_t)(I.nz + 2) * (cs + sizeof(T) + sizeof(int)) + 64; }

  hipError_t x1(const void* const* in, void* const* out, bool nz) {
    StageArgs a = base(IT_X1, nz, 0);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_tr_x1_r2c<T>, "dft_x1", a, max_over(sh_x1), st, tm);
  }
  hipError_t x2(void* const* io, bool nz, int inv) {
    StageArgs a = base(IT_X2, nz, inv);
    for (int i = 0; i < n; ++i) {
      a.in[i] = io[i];
      a.out[i] = io[i];
    }
    return launch(k_tr_x2<T>, inv ? "idft_x2" : "dft_x2", a, max_over(sh_x2), st, tm);
  }
  hipError_t c2r(const void* const* in, void* const* out, bool nz) {
    StageArgs a = base(IT_C2R, nz, 0);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_tr_c2r_k1<T>, "idft_x1_c2r", a, max_over(sh_x1), st, tm);
  }
  hipError_t zfft(void* const* io, int inv) {
    StageArgs a = base(IT_LINES, true, inv);
    for (int i = 0; i < n; ++i) {
      a.in[i] = io[i];
      a.out[i] = io[i];
    }
    return launch(k_line_fft<T>, inv ? "idft_z" : "dft_z", a, max_over(sh_z), st, tm);
  }
  hipError_t a2(const void* const* in, void* const* out) {
    StageArgs a = base(IT_LINES, false, 0);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_line_a2<T, G>, "deconv_pad_fft", a, max_over(sh_m), st, tm);
  }
  hipError_t a2t(const void* const* in, void* const* out) {
    StageArgs a = base(IT_LINES, false, 0);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_line_a2t<T, G>, "ifft_pick_deconv", a, max_over(sh_m), st, tm);
  }
  hipError_t interp(const void* const* in, void* const* out, int mode) {
    StageArgs a = base(IT_LINES, true, mode);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_line_interp<T, G>, "interp", a, max_over(sh_m), st, tm);
  }
  hipError_t spread(const void* const* in, void* const* out, int mode) {
    StageArgs a = base(IT_LINES, true, mode);
    for (int i = 0; i < n; ++i) {
      a.in[i] = in[i];
      a.out[i] = out[i];
    }
    return launch(k_line_spread<T, G>, "spread", a, max_over(sh_spread), st, tm);
  }
};

#define PAT_TRY(x)                  \
  do {                              \
    hipError_t e_ = (x);            \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T, typename G>
hipError_t run_op_t(Op op, int n, const Inst* h, const Inst* const* d, const void* const* in,
                    void* const* out, void* const* ws, uint32_t* counters, hipStream_t st, StageTimer* tm) {
  Runner<T, G> r{n, h, d, counters, 0, st, tm};
  void* bg[kMaxBatch];
  void* bu[kMaxBatch];
  void* bf[kMaxBatch];
  for (int i = 0; i < n; ++i) {
    char* w = static_cast<char*>(ws[i]);
    bg[i] = w + h[i].off_g;
    bu[i] = w + h[i].off_u;
    bf[i] = w + h[i].off_f;
  }
  if (counters) {
    if (tm) tm->begin("zero_counters", st);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counters, kNumCounters);
    PAT_TRY(hipGetLastError());
    if (tm) tm->end(st);
  }
  switch (op) {
    case OP_R:
    case OP_AT:
      PAT_TRY(r.x1(in, bg, false));
      PAT_TRY(r.x2(bg, false, 0));
      PAT_TRY(r.a2(bg, bu));
      PAT_TRY(r.interp(bu, bf, op == OP_R ? 0 : 1));
      PAT_TRY(r.zfft(bf, 1));
      PAT_TRY(r.x2(bf, true, 1));
      PAT_TRY(r.c2r(bf, out, true));
      break;
    case OP_RT:
    case OP_A:
      PAT_TRY(r.x1(in, bf, true));
      PAT_TRY(r.x2(bf, true, 0));
      PAT_TRY(r.zfft(bf, 0));
      PAT_TRY(r.spread(bf, bu, op == OP_RT ? 0 : 1));
      PAT_TRY(r.a2t(bu, bg));
      PAT_TRY(r.x2(bg, false, 1));
      PAT_TRY(r.c2r(bg, out, false));
      break;
  }
  return hipSuccess;
}

}  // namespace

hipError_t run_op(int prec, Op op, int n, const Inst* hinst, const Inst* const* dinst, const void* const* in,
                  void* const* out, void* const* ws, uint32_t* counters, hipStream_t stream, StageTimer* timer) {
  switch (prec) {
    case PREC_F64:
      return run_op_t<double, cx<double>>(op, n, hinst, dinst, in, out, ws, counters, stream, timer);
    case PREC_F32:
      return run_op_t<float, cx<float>>(op, n, hinst, dinst, in, out, ws, counters, stream, timer);
    case PREC_BF16:
      return run_op_t<float, bf2>(op, n, hinst, dinst, in, out, ws, counters, stream, timer);
  }
  return hipErrorInvalidValue;
}

hipError_t run_interp(int prec, const Inst& hinst, const Inst* dinst, const void* grid, void* out, hipStream_t stream,
                      StageTimer* timer) {
  const Inst* d[1] = {dinst};
  const void* in[1] = {grid};
  void* o[1] = {out};
  switch (prec) {
    case PREC_F64: {
      Runner<double, cx<double>> r{1, &hinst, d, nullptr, 0, stream, timer};
      return r.interp(in, o, 0);
    }
    case PREC_F32: {
      Runner<float, cx<float>> r{1, &hinst, d, nullptr, 0, stream, timer};
      return r.interp(in, o, 0);
    }
    case PREC_BF16: {
      Runner<float, bf2> r{1, &hinst, d, nullptr, 0, stream, timer};
      return r.interp(in, o, 0);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace pat
