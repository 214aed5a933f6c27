// CDNA4 (gfx950) kernels of the NUFFT-based planar photoacoustic
// reconstruction.  Every kernel runs 256-thread workgroups over a list of work
// items (instance, tile or group of lines); items come either one per
// workgroup or from a device work counter drained by a persistent grid (the
// batched form).
//
// Stages (a1 .. a5 are the steps of R as pat.h lists them under
// pat_reconstruct; see pat.h for the operators they compose):
//   k_tr_x1_r2c   DFT over the first detector axis, real input, half spectrum
//   k_tr_x2       DFT over the second detector axis (either direction)
//   k_tr_c2r_k1   inverse DFT over the first axis from the half spectrum, real part
//   k_tr_*_pipe   the three above as software pipelines (one FP32 instance)
//   k_line_fft    DFT along contiguous lines (depth axis)
//   k_line_a2     deconvolve by 1/Psi, centre, zero-pad to c*nt, FFT (eq. nufft-c)
//                 (k_line_a2_pipe: its software pipeline, c = 2, sizes fixed
//                 at compile time)
//   k_line_a2t    its transpose: inverse FFT, pick, multiply by 1/Psi
//                 (k_line_a2t_pipe: likewise)
//   k_line_interp type-2 interpolation with 2cK Kaiser-Bessel taps (eq. nufft-a)
//                 and the Jacobian weight (eq. fft-0) (k_line_interp_stream:
//                 persistent, the next line group streamed into registers)
//   k_line_spread its transpose (type-1), gathered per grid cell over the
//                 monotone node list of the line: no atomics, deterministic
//                 (k_line_spread_w: one line per wavefront, segmented sums
//                 across lanes, FP32)
//   k_line_nufft2 a2 + a3 + inverse depth DFT fused per line group in LDS
//                 (k_line_nufft2_pipe: its software pipeline for c = 2;
//                 k_line_nufft2_pipe_c: the same for sizes fixed at compile
//                 time; k_line_nufft2_mirror: R on 3D plans with nz = m/4,
//                 the lines of an item in mirror pairs sharing node windows)
//   k_line_nufft1 depth DFT + spreading + transposed a2 fused per line in LDS
//                 (k_line_nufft1_c: sizes fixed at compile time;
//                 k_line_nufft1_w: one line per wavefront, FP32)
// The fused kernels never store the oversampled grid; the staged ones do
// (bf16 grid option, long grid lines, and the stand-alone a3 / spreading
// entry points).
//
// Uniform FFTs are in-place decimation-in-frequency mixed-radix transforms in
// LDS; bin k ends at position perm[k] (a table built by the host plan).  Two
// instantiations exist: radices 2/4/8 with shift arithmetic (all lengths
// powers of two), and the general one (odd primes up to 23).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>

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

template <typename T>
struct Deg;
template <>
struct Deg<float> {
  static constexpr int v = kPolyDegF;
};
template <>
struct Deg<double> {
  static constexpr int v = kPolyDegD;
};

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
// buf[b*bs + e*es].  BF selects the thread mapping: butterfly index fastest
// (contiguous lines) or transform index fastest (column tiles).

template <typename T, int R>
__device__ __forceinline__ void dft_pow2(cx<T>* v) {
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
  } else if constexpr (R == 16) {
    // two 8-point DFTs of the even and odd samples, odd outputs turned by
    // exp(-2 pi i d / 16)
    cx<T> e[8], o[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      e[r] = v[2 * r];
      o[r] = v[2 * r + 1];
    }
    dft_pow2<T, 8>(e);
    dft_pow2<T, 8>(o);
    const T c1 = T(0.92387953251128675612818318939678829), s1 = T(0.38268343236508977172845998403039887);
    const T h = T(0.70710678118654752440084436210484904);
    const T cs[8] = {T(1), c1, h, s1, T(0), -s1, -h, -c1};
    const T sn[8] = {T(0), s1, h, c1, T(1), c1, h, s1};
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const cx<T> t = mk(o[d].x * cs[d] + o[d].y * sn[d], o[d].y * cs[d] - o[d].x * sn[d]);
      v[d] = cadd(e[d], t);
      v[d + 8] = csub(e[d], t);
    }
  } else {
    static_assert(R == 8, "radix");
    const T h = T(0.70710678118654752440084436210484904);
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft_pow2<T, 4>(e);
    dft_pow2<T, 4>(o);
    // o[d] *= exp(-2 pi i d / 8)
    const cx<T> o1 = mk(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    const cx<T> o2 = cmi(o[2]);
    const cx<T> o3 = mk(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// The roots exp(-2 pi i q / R) of an odd prime R as compile-time constants:
// cos and sin of 2 pi q / R from Taylor series in double on the angle
// reduced to [-pi/4, pi/4] by quarter turns (error below 1e-16).
struct RootTable {
  double c[24], s[24];
};
constexpr RootTable make_roots(int R) {
  RootTable t{};
  for (int q = 0; q < R; ++q) {
    const int k = (8 * q + R) / (2 * R);  // nearest multiple of a quarter turn
    const double x = 3.14159265358979323846 * (double)(4 * q - k * R) / (2.0 * R);
    double sn = x, cs = 1.0, ts = x, tc = 1.0;
    for (int i = 1; i < 14; ++i) {
      ts *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
      tc *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
      sn += ts;
      cs += tc;
    }
    switch (k & 3) {
      case 0: t.c[q] = cs; t.s[q] = sn; break;
      case 1: t.c[q] = -sn; t.s[q] = cs; break;
      case 2: t.c[q] = -cs; t.s[q] = -sn; break;
      default: t.c[q] = sn; t.s[q] = -cs; break;
    }
  }
  return t;
}
template <int R>
struct Roots {
  static constexpr RootTable t = make_roots(R);
};
// the same tables in constant memory, for the larger primes' rolled loops
__constant__ RootTable kRoots11 = make_roots(11);
__constant__ RootTable kRoots13 = make_roots(13);
__constant__ RootTable kRoots17 = make_roots(17);
__constant__ RootTable kRoots19 = make_roots(19);
__constant__ RootTable kRoots23 = make_roots(23);
template <int R>
__device__ __forceinline__ const RootTable& root_table() {
  if constexpr (R == 11) return kRoots11;
  else if constexpr (R == 13) return kRoots13;
  else if constexpr (R == 17) return kRoots17;
  else if constexpr (R == 19) return kRoots19;
  else return kRoots23;
}

// Odd-prime butterfly, all in registers: outputs d and R - d together, with
// a_r = x_r + x_{R-r}, b_r = x_r - x_{R-r} (r = 1 .. H) and theta = 2 pi r d / R,
//   X_d = x_0 + sum_r a_r cos(theta) - i sum_r b_r sin(theta),
//   X_{R-d} = x_0 + sum_r a_r cos(theta) + i sum_r b_r sin(theta),
// a quarter of the direct DFT's multiply-adds.  Up to R = 7 the cosines and
// sines are compile-time constants (both loops unroll, so every index is
// known); only the twiddles of the stage, exp(-2 pi i j d / Li), come from
// the table.
template <typename T, int R, typename Ptr>
__device__ __forceinline__ void bfly_prime(Ptr p, int st, int j, int tws, const cx<T>* __restrict__ tw, int L) {
  constexpr int H = (R - 1) / 2;
  (void)L;
  const cx<T> x0 = ldx(p);
  cx<T> av[H + 1], bv[H + 1];
  cx<T> X0 = x0;
#pragma unroll
  for (int r = 1; r <= H; ++r) {
    const cx<T> u = ldx(p + r * st), v = ldx(p + (R - r) * st);
    av[r] = cadd(u, v);
    bv[r] = csub(u, v);
    X0 = cadd(X0, av[r]);
  }
  stx(p, X0);
  auto emit = [&](int d, cx<T> A, cx<T> B) {
    cx<T> Xd = mk(A.x + B.y, A.y - B.x), Xm = mk(A.x - B.y, A.y + B.x);
    if (j) {
      Xd = cmul(Xd, tw[j * d * tws]);
      Xm = cmul(Xm, tw[j * (R - d) * tws]);
    }
    stx(p + d * st, Xd);
    stx(p + (R - d) * st, Xm);
  };
  if constexpr (R <= 7) {
#pragma unroll
    for (int d = 1; d <= H; ++d) {
      cx<T> A = x0, B = mk(T(0), T(0));
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        const int q = (r * d) % R;
        const T c = T(Roots<R>::t.c[q]), sn = T(Roots<R>::t.s[q]);
        A.x += av[r].x * c;
        A.y += av[r].y * c;
        B.x += bv[r].x * sn;
        B.y += bv[r].y * sn;
      }
      emit(d, A, B);
    }
  } else {
    // the larger primes: one output pair at a time (a rolled loop keeps the
    // register footprint of a fully unrolled butterfly out of the kernel),
    // the roots read at a wave-uniform index from constant memory
    const RootTable& rt = root_table<R>();
#pragma unroll 1
    for (int d = 1; d <= H; ++d) {
      cx<T> A = x0, B = mk(T(0), T(0));
      int q = 0;
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        q += d;
        q -= q >= R ? R : 0;
        const T c = T(rt.c[q]), sn = T(rt.s[q]);
        A.x += av[r].x * c;
        A.y += av[r].y * c;
        B.x += bv[r].x * sn;
        B.y += bv[r].y * sn;
      }
      emit(d, A, B);
    }
  }
}

// Element access through a pointer of any address space (field by field:
// the implicit copy operations of cx bind to generic-address objects only).
template <typename P>
__device__ __forceinline__ auto ldx(P p) {
  return mk(p->x, p->y);
}
template <typename P, typename T>
__device__ __forceinline__ void stx(P p, cx<T> v) {
  p->x = v.x;
  p->y = v.y;
}

// v[d] *= w^d for d = 1 .. R-1 from the one table twiddle w of a butterfly
// (w = exp(-2 pi i j / Li)); the powers come from a product tree at most
// three products deep.
template <typename T, int R>
__device__ __forceinline__ void twiddle_pow2(cx<T>* v, cx<T> w1) {
  cx<T> w[R];
  w[1] = w1;
  if constexpr (R >= 4) {
    w[2] = cmul(w[1], w[1]);
    w[3] = cmul(w[2], w[1]);
  }
  if constexpr (R == 8) {
    w[4] = cmul(w[2], w[2]);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  }
#pragma unroll
  for (int d = 1; d < R; ++d) v[d] = cmul(v[d], w[d]);
}

// With PADL > 0 the scratch is padded: element i sits at i + (i >> PADL), one
// spare slot after every 2^PADL points, so that the strided butterfly
// accesses of the later stages (lanes 2^PADL points apart) spread over the
// LDS banks (power-of-two radices only).
// (NT: the threads of the workgroup)
template <typename T, int R, bool P2, bool BF, typename Ptr = cx<T>*, int PADL = 0, int NT = kBlock>
__device__ __forceinline__ void fft_stage(Ptr buf, int Li, int L, const cx<T>* __restrict__ tw, int nb,
                                          int bs, int es) {
  static_assert(PADL == 0 || R == 2 || R == 4 || R == 8 || R == 16, "padded scratch: power-of-two radices");
  const int sub = Li / R;
  const int tws = L / Li;
  const int nbf = L / R;
  const int total = nbf * nb;
  int lsub = 0, lnbf = 0, lnb = 0;
  if constexpr (P2) {
    lsub = __builtin_ctz((unsigned)sub);
    lnbf = __builtin_ctz((unsigned)nbf);
    lnb = __builtin_ctz((unsigned)nb);
  }
  // (one butterfly per loop trip, not unrolled: each has ILP of its own, and
  // two in flight would double the stage's register footprint)
#pragma unroll 1
  for (int id = threadIdx.x; id < total; id += NT) {
    int b, bf;
    if constexpr (BF) {
      if constexpr (P2) {
        bf = id & (nbf - 1);
        b = id >> lnbf;
      } else {
        b = id / nbf;
        bf = id - b * nbf;
      }
    } else {
      if constexpr (P2) {
        b = id & (nb - 1);
        bf = id >> lnb;
      } else {
        bf = id / nb;
        b = id - bf * nb;
      }
    }
    int blk, j;
    if constexpr (P2) {
      blk = bf >> lsub;
      j = bf & (sub - 1);
    } else {
      blk = bf / sub;
      j = bf - blk * sub;
    }
    const int i0 = b * bs + (blk * Li + j) * es;
    Ptr p = buf + i0;
    const int st = sub * es;
    // (strides that are multiples of 2^PADL keep a constant padded stride)
    const int pst = PADL > 0 && st % (1 << PADL) == 0 ? st + (st >> PADL) : 0;
    Ptr pp = PADL > 0 ? buf + (i0 + (i0 >> PADL)) : p;
    auto at = [&](int r) {
      if constexpr (PADL > 0) {
        const int i = i0 + r * st;
        return pst ? pp + r * pst : buf + (i + (i >> PADL));
      }
      return p + r * st;
    };
    if constexpr (R == 2 || R == 4 || R == 8) {
      cx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = ldx(at(r));
      dft_pow2<T, R>(v);
      // (the last stage, sub = 1, has j = 0 and no twiddles)
      if (sub > 1) twiddle_pow2<T, R>(v, tw[j * tws]);
#pragma unroll
      for (int r = 0; r < R; ++r) stx(at(r), v[r]);
    } else {
      bfly_prime<T, R>(p, st, j, tws, tw, L);
    }
  }
}

// tw: the L roots exp(-2 pi i k / L) of this transform (in LDS in every kernel)
// One general-radix stage as a function of its own: called once per stage,
// it gets its own register allocation instead of sharing one with every
// other radix of the build.
template <typename T, int R, bool BF>
__device__ __noinline__ void fft_stage_fn(cx<T>* buf, int Li, int L, const cx<T>* __restrict__ tw, int nb, int bs,
                                          int es) {
  typedef __attribute__((address_space(3))) cx<T>* LdsPtr;
  fft_stage<T, R, false, BF, LdsPtr>((LdsPtr)buf, Li, L, tw, nb, bs, es);
}

// RS selects the radix set a kernel build carries: 0 the powers of two (2, 4,
// 8 with shift arithmetic), 7 the radices up to 7, 23 every radix the plans
// emit.  A build with fewer radices keeps fewer registers live.
template <typename T, int RS, bool BF>
__device__ void fft_lds(cx<T>* buf, const FftDesc& d, const cx<T>* __restrict__ tw, int nb, int bs, int es) {
  constexpr bool P2 = RS == 0;
  const int L = d.L;
  int Li = L;
  for (int s = 0; s < d.nst; ++s) {
    const int R = d.rad[s];
    if constexpr (P2) {
      if (R == 8) fft_stage<T, 8, P2, BF>(buf, Li, L, tw, nb, bs, es);
      else if (R == 4) fft_stage<T, 4, P2, BF>(buf, Li, L, tw, nb, bs, es);
      else fft_stage<T, 2, P2, BF>(buf, Li, L, tw, nb, bs, es);
    } else {
      switch (R) {
        case 2: fft_stage_fn<T, 2, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 3: fft_stage_fn<T, 3, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 4: fft_stage_fn<T, 4, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 5: fft_stage_fn<T, 5, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 7: fft_stage_fn<T, 7, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 8: fft_stage_fn<T, 8, BF>(buf, Li, L, tw, nb, bs, es); break;
        case 11:
          if constexpr (RS >= 11) fft_stage_fn<T, 11, BF>(buf, Li, L, tw, nb, bs, es);
          break;
        case 13:
          if constexpr (RS >= 13) fft_stage_fn<T, 13, BF>(buf, Li, L, tw, nb, bs, es);
          break;
        case 17:
          if constexpr (RS >= 17) fft_stage_fn<T, 17, BF>(buf, Li, L, tw, nb, bs, es);
          break;
        case 19:
          if constexpr (RS >= 19) fft_stage_fn<T, 19, BF>(buf, Li, L, tw, nb, bs, es);
          break;
        case 23:
          if constexpr (RS >= 23) fft_stage_fn<T, 23, BF>(buf, Li, L, tw, nb, bs, es);
          break;
        default: break;  // the host plan only emits the radices above
      }
    }
    __syncthreads();
    Li /= R;
  }
}

// Natural (frequency) index of the in-place DIF output at position pos: the
// digits of pos, most significant first, are those of k, least significant
// first (radices of the stages in order); power-of-two radices.
__device__ __forceinline__ int dif_natural_p2(const FftDesc& d, int pos) {
  int k = 0, sh = 0, lspan = __builtin_ctz((unsigned)d.L);
  for (int s = 0; s < d.nst; ++s) {
    const int lr = __builtin_ctz((unsigned)d.rad[s]);
    lspan -= lr;
    k += (pos >> lspan) << sh;
    pos &= (1 << lspan) - 1;
    sh += lr;
  }
  return k;
}

// The inverse of dif_natural_p2: the position of natural index k in the
// in-place DIF output (its digits, least significant first, become the
// position's digits, most significant first).
__device__ __forceinline__ int dif_position_p2(const FftDesc& d, int k) {
  int pos = 0, lspan = __builtin_ctz((unsigned)d.L);
  for (int s = 0; s < d.nst; ++s) {
    const int lr = __builtin_ctz((unsigned)d.rad[s]);
    lspan -= lr;
    pos += (k & (d.rad[s] - 1)) << lspan;
    k >>= lr;
  }
  return pos;
}

// The last stage (sub = 1, no twiddles) of a power-of-two DIF transform,
// handing each butterfly's R outputs (positions blk*R + r) to
// sink(b, blk, v) instead of writing them back.
template <typename T, int R, bool BF, int PADL = 0, int NT = kBlock, typename Sink>
__device__ __forceinline__ void fft_last_stage_p2(const cx<T>* buf, int L, int nb, int bs, int es, Sink sink) {
  const int nbf = L / R;
  const int lnbf = __builtin_ctz((unsigned)nbf), lnb = __builtin_ctz((unsigned)nb);
  for (int id = threadIdx.x; id < nbf * nb; id += NT) {
    int b, blk;
    if constexpr (BF) {
      blk = id & (nbf - 1);
      b = id >> lnbf;
    } else {
      b = id & (nb - 1);
      blk = id >> lnb;
    }
    // (padded: a run of R <= 2^PADL points from a multiple of R stays in one
    // padded block when es = 1)
    const int i0 = b * bs + blk * R * es;
    const cx<T>* p = buf + (PADL > 0 ? i0 + (i0 >> PADL) : i0);
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (PADL > 0) {
        const int i = i0 + r * es;
        v[r] = es == 1 && R <= (1 << PADL) ? p[r] : buf[i + (i >> PADL)];
      } else {
        v[r] = p[r * es];
      }
    }
    dft_pow2<T, R>(v);
    sink(b, blk, v);
  }
}

// The first stage (Li = L) of a power-of-two DIF transform whose inputs come
// from src(b, pos) rather than buf: butterfly j of transform b takes the
// positions j + r*sub, and its twiddled outputs go to buf.
template <typename T, int R, bool BF, typename Src>
__device__ __forceinline__ void fft_first_stage_p2(cx<T>* buf, int L, const cx<T>* __restrict__ tw, int nb, int bs,
                                                   int es, Src src) {
  const int sub = L / R;
  const int lsub = __builtin_ctz((unsigned)sub), lnb = __builtin_ctz((unsigned)nb);
  for (int id = threadIdx.x; id < sub * nb; id += kBlock) {
    int b, j;
    if constexpr (BF) {
      j = id & (sub - 1);
      b = id >> lsub;
    } else {
      b = id & (nb - 1);
      j = id >> lnb;
    }
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src(b, j + r * sub);
    dft_pow2<T, R>(v);
    if (sub > 1) twiddle_pow2<T, R>(v, tw[j]);
    cx<T>* p = buf + b * bs + j * es;
#pragma unroll
    for (int r = 0; r < R; ++r) p[r * sub * es] = v[r];
  }
}

// fft_lds for power-of-two lengths whose inputs come from src(b, pos) (first
// stage, see fft_first_stage_p2) and whose result goes to sink(b, blk, v[R])
// (last stage, see fft_last_stage_p2).
template <typename T, bool BF, typename Src, typename Sink>
__device__ void fft_lds_p2_src_sink(cx<T>* buf, const FftDesc& d, const cx<T>* __restrict__ tw, int nb, int bs,
                                    int es, Src src, Sink sink) {
  const int L = d.L;
  if (d.nst == 1) {
    for (int id = threadIdx.x; id < L * nb; id += kBlock) {
      const int b = id / L, pos = id - b * L;
      buf[b * bs + pos * es] = src(b, pos);
    }
  } else {
    const int R0 = d.rad[0];
    if (R0 == 8) fft_first_stage_p2<T, 8, BF>(buf, L, tw, nb, bs, es, src);
    else if (R0 == 4) fft_first_stage_p2<T, 4, BF>(buf, L, tw, nb, bs, es, src);
    else fft_first_stage_p2<T, 2, BF>(buf, L, tw, nb, bs, es, src);
  }
  __syncthreads();
  int Li = d.nst == 1 ? L : L / d.rad[0];
  for (int s = d.nst == 1 ? 0 : 1; s + 1 < d.nst; ++s) {
    const int R = d.rad[s];
    if (R == 8) fft_stage<T, 8, true, BF>(buf, Li, L, tw, nb, bs, es);
    else if (R == 4) fft_stage<T, 4, true, BF>(buf, Li, L, tw, nb, bs, es);
    else fft_stage<T, 2, true, BF>(buf, Li, L, tw, nb, bs, es);
    __syncthreads();
    Li /= R;
  }
  const int R = d.rad[d.nst - 1];
  if (R == 8) fft_last_stage_p2<T, 8, BF>(buf, L, nb, bs, es, sink);
  else if (R == 4) fft_last_stage_p2<T, 4, BF>(buf, L, nb, bs, es, sink);
  else fft_last_stage_p2<T, 2, BF>(buf, L, nb, bs, es, sink);
  __syncthreads();
}

// Radix plan of 2^E points known at compile time, by the host plan's rule:
// radix 8 while it divides, ending in 4 (E mod 3 = 2), 4 and 4 (E mod 3 = 1,
// E >= 4), or 2 (E = 1).  With L16 the plan of 2^(E-4) points is followed by
// one radix-16 stage instead (used where the output order is the kernel's
// own, not the host's permutation table).  With every length and stage a
// constant, the stage loops, index shifts and output positions fold at
// compile time.
template <int E, bool L16 = false>
struct P2Plan {
  static constexpr int n8 = E / 3, rem = E % 3;
  static constexpr int nst = L16 ? P2Plan<(L16 ? E - 4 : 1)>::nst + 1 : rem == 0 ? n8 : n8 + 1;
  static constexpr int rad(int s) {
    if (L16) return s + 1 == nst ? 16 : P2Plan<(L16 ? E - 4 : 1)>::rad(s);
    return rem == 0 ? 8 : rem == 2 ? (s < n8 ? 8 : 4) : n8 > 0 ? (s < n8 - 1 ? 8 : 4) : 2;
  }
  static constexpr int lbits(int s) { return rad(s) == 16 ? 4 : rad(s) == 8 ? 3 : rad(s) == 4 ? 2 : 1; }
  // log2 of the span Li that stage s works on
  static constexpr int lspan(int s) { return s == 0 ? E : lspan(s - 1) - lbits(s - 1); }
  // natural index of the output at position pos (digit reversal of the plan)
  static __device__ __forceinline__ int natural(int pos) {
    int k = 0, sh = 0;
#pragma unroll
    for (int s = 0; s < nst; ++s) {
      const int lo = lspan(s) - lbits(s);
      k += ((pos >> lo) & ((1 << lbits(s)) - 1)) << sh;
      sh += lbits(s);
    }
    return k;
  }
};
static_assert(P2Plan<10>::nst == 4 && P2Plan<10>::rad(0) == 8 && P2Plan<10>::rad(2) == 4, "plan of 1024");
static_assert(P2Plan<8>::nst == 3 && P2Plan<8>::rad(2) == 4 && P2Plan<9>::rad(2) == 8, "plans of 256, 512");
// the fused type-2 kernel ends its transforms in one radix-16 stage (which
// has no twiddles): the depth FFT from 64 points on, the grid FFT where the
// plan before it still opens with the radix-8 stage its pipeline needs
constexpr bool p2_l16_z(int e) { return e >= 6; }
constexpr bool p2_l16_m(int e) { return e >= 9; }
static_assert(P2Plan<10, true>::nst == 3 && P2Plan<10, true>::rad(1) == 8 && P2Plan<10, true>::rad(2) == 16 &&
                  P2Plan<7, true>::nst == 2 && P2Plan<7, true>::rad(0) == 8 && P2Plan<7, true>::lspan(1) == 4,
              "plans ending in radix 16");

// Stages S .. nst - 2 (twiddled, in place) of the compile-time plan of 2^E
// points on nb lines of stride 2^E, one block barrier after each.
// (PADL: the padded scratch of fft_stage.)
template <typename T, int E, int S, bool L16 = false, int PADL = 0, int NT = kBlock>
__device__ __forceinline__ void p2_stages(cx<T>* buf, const cx<T>* __restrict__ tw, int nb) {
  using Pl = P2Plan<E, L16>;
  if constexpr (S + 1 < Pl::nst) {
    fft_stage<T, Pl::rad(S), true, true, cx<T>*, PADL, NT>(buf, 1 << Pl::lspan(S), 1 << E, tw, nb, 1 << E, 1);
    __syncthreads();
    p2_stages<T, E, S + 1, L16, PADL, NT>(buf, tw, nb);
  }
}

// Every stage (in place, each followed by a block barrier) of the
// compile-time plan of 2^E points: fft_lds with the sizes fixed.
template <typename T, int E, bool BF, int S = 0>
__device__ __forceinline__ void p2_fft(cx<T>* buf, const cx<T>* __restrict__ tw, int nb, int bs, int es) {
  using Pl = P2Plan<E>;
  if constexpr (S < Pl::nst) {
    fft_stage<T, Pl::rad(S), true, BF>(buf, 1 << Pl::lspan(S), 1 << E, tw, nb, bs, es);
    __syncthreads();
    p2_fft<T, E, BF, S + 1>(buf, tw, nb, bs, es);
  }
}

// fft_lds for power-of-two lengths whose result goes to sink(b, blk, v[R])
// from the last stage (see fft_last_stage_p2) rather than back into buf.
template <typename T, bool BF, typename Sink>
__device__ void fft_lds_p2_sink(cx<T>* buf, const FftDesc& d, const cx<T>* __restrict__ tw, int nb, int bs, int es,
                                Sink sink) {
  const int L = d.L;
  int Li = L;
  for (int s = 0; s + 1 < d.nst; ++s) {
    const int R = d.rad[s];
    if (R == 8) fft_stage<T, 8, true, BF>(buf, Li, L, tw, nb, bs, es);
    else if (R == 4) fft_stage<T, 4, true, BF>(buf, Li, L, tw, nb, bs, es);
    else fft_stage<T, 2, true, BF>(buf, Li, L, tw, nb, bs, es);
    __syncthreads();
    Li /= R;
  }
  const int R = d.rad[d.nst - 1];
  if (R == 8) fft_last_stage_p2<T, 8, BF>(buf, L, nb, bs, es, sink);
  else if (R == 4) fft_last_stage_p2<T, 4, BF>(buf, L, nb, bs, es, sink);
  else fft_last_stage_p2<T, 2, BF>(buf, L, nb, bs, es, sink);
  __syncthreads();
}

// quotient and remainder by a length that is a power of two in the P2 path
template <bool P2>
__device__ __forceinline__ void divmod(int e, int L, int* q, int* r) {
  if constexpr (P2) {
    const int s = __builtin_ctz((unsigned)L);
    *q = e >> s;
    *r = e & (L - 1);
  } else {
    *q = e / L;
    *r = e - *q * L;
  }
}


// Issues U independent loads per thread before storing them, so that each
// thread keeps several memory requests in flight:
// for e in [tid, total) step kBlock:  st(e, ld(e)).
template <int U, typename Ld, typename St>
__device__ __forceinline__ void copy_batched(int total, Ld ld, St st) {
  using V = decltype(ld(0));
  for (int e0 = threadIdx.x; e0 < total; e0 += U * kBlock) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kBlock;
      if (e < total) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * kBlock;
      if (e < total) st(e, v[u]);
    }
  }
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
  uint32_t* counter;  // persistent queue, or nullptr: items blockIdx.x + i gridDim.x
  int32_t item_slot;  // with a counter: byte offset of the item slot in dynamic LDS
  int32_t len_nz;     // transverse passes: lines have nz (else nt) samples
  int32_t mode;       // FFT direction (0 forward, 1 inverse) / interp, spread mode
  int32_t pair_ok;    // pc holds every instance's mirrored tap-pair polynomials
  // per tap pair p (taps t = p and taps-1-p): even part (powers x^0, x^2, ...)
  // then odd part (x^1, x^3, ...) of tap p's polynomial, in the compute type
  alignas(8) uint32_t pc[kPolyWords];
};

// Copies the L roots of one FFT length from the instance table into LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cx<T>* dst, const Inst& I, const FftDesc& d) {
  const cx<T>* src = static_cast<const cx<T>*>(I.tw) + d.tw;
  for (int e = threadIdx.x; e < d.L; e += kBlock) dst[e] = src[e];
}

// ---------------------------------------------------------------------------
// Kaiser-Bessel interpolation kernel.  With s = sqrt(K^2 - u^2), |u| <= K,
//   Psi_hat(u) I0(alpha K) / (2 e^{alpha K}) = e^{alpha (s - K)} (1 - e^{-2 alpha s}) / (2 s)
// (the transform of Section 3.2 with the large factor e^{alpha K} / I0(alpha K)
// moved into the deconvolution table), limit alpha e^{-alpha K} at s -> 0.
// Direct evaluation; the tap loops normally use the per-tap polynomials the
// host plan fitted to this function instead.

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

// tap of a node whose offset is x = 2 (delta - cK) + 1, from its coefficient row
template <typename T>
__device__ __forceinline__ T tap_poly(const T* __restrict__ c, T x) {
  constexpr int D = Deg<T>::v;
  T w = c[D];
#pragma unroll
  for (int d = D - 1; d >= 0; --d) w = w * x + c[d];
  return w;
}

// First tap of a node at grid position xc = c nu: j0 = floor(xc - cK) + 1,
// with d = xc - j0 - cK + 1 - 1 = (fractional part of xc) - 1 returned; the
// node's tap offset is x = 2 d + 1 in [-1, 1).  Formed in double without
// contraction (the subtractions see the rounded xc).  Where the paired taps
// are used, the window of -nup is never formed from -xc but as the mirror
// image of +nup's (interp_pair, spread_node, spread_line_wave): near 0,
// rounding in xc - cK can make the direct form pick the window one end tap
// over, and the interpolation and the spreading must agree on the window.
__device__ __forceinline__ double tap_origin(double xc, double ck, int* j0) {
#pragma clang fp contract(off)
  const double f = floor(xc - ck);
  *j0 = (int)f + 1;
  return xc - f - 1.0 - ck;
}

// exp(-i pi nu), argument reduced in double to r in [-1, 1].  Double: the
// library sincospi.  Float: r = s + q/2 with |s| <= 1/4 and q = rint(2r);
// sin and cos of pi s from polynomials in s^2 fitted by least squares
// (gen_sincospi.py; largest error below 1e-7 when evaluated in float),
// rotated by q quarter turns.
template <typename T>
__device__ __forceinline__ cx<T> phase_mpi(double nu) {
  const double r = nu - 2.0 * rint(0.5 * nu);
  T s, c;
  m_sincospi((T)r, &s, &c);
  return mk(c, -s);
}
template <>
__device__ __forceinline__ cx<float> phase_mpi<float>(double nu) {
  const float r = (float)(nu - 2.0 * rint(0.5 * nu));
  const float q = rintf(2.0f * r);
  const float s = fmaf(-0.5f, q, r);
  const float u = s * s;
  float ps = fmaf(u, -0.5890768766403198f, 2.549767017364502f);
  ps = fmaf(u, ps, -5.167707920074463f);
  ps = fmaf(u, ps, 3.1415927410125732f);
  const float sn = s * ps;
  float pc = fmaf(u, 0.23132924735546112f, -1.335044503211975f);
  pc = fmaf(u, pc, 4.058707237243652f);
  pc = fmaf(u, pc, -4.934802055358887f);
  const float cs = fmaf(u, pc, 1.0f);
  // sin(pi (s + q/2)), cos(pi (s + q/2)) for q mod 4 = 0, 1, 2, 3:
  // (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn)
  const int qi = (int)q & 3;
  float sv = (qi & 1) ? cs : sn;
  float cv = (qi & 1) ? sn : cs;
  if (qi == 1 || qi == 2) cv = -cv;
  if (qi >= 2) sv = -sv;
  return mk(cv, -sv);
}

// nu+ = sqrt(A) and 1/nu in double from a float estimate and one Newton step
// (relative error ~1e-14, far cheaper than the correctly rounded operations).
__device__ __forceinline__ double sqrt_nt(double A) {
  const float s0 = __builtin_amdgcn_sqrtf((float)A);
  if (s0 == 0.0f) return 0.0;
  const double s = (double)s0;
  return fma(fma(-s, s, A), (double)(0.5f * __builtin_amdgcn_rcpf(s0)), s);
}
__device__ __forceinline__ double rcp_nt(double v) {
  const double y = (double)__builtin_amdgcn_rcpf((float)v);
  return y * fma(-v, y, 2.0);
}

// The TAPS tap weights of a node with offset x = 2 (delta - cK) + 1, from the
// mirrored pairs in the kernel arguments: tap taps-1-t at x equals tap t at -x
// (the kernel is even), so each pair costs one even and one odd polynomial
// in x^2 on workgroup-uniform coefficients.
template <typename T, int TAPS>
__device__ __forceinline__ void tap_weights_pairs(const StageArgs& a, T x, T* w) {
  constexpr int D = Deg<T>::v, NE = D / 2 + 1, NO = (D + 1) / 2, PW = NE + NO;
  const T* pc = reinterpret_cast<const T*>(a.pc);
  const T y = x * x;
#pragma unroll
  for (int p = 0; p < TAPS / 2; ++p) {
    T e = pc[p * PW + NE - 1];
#pragma unroll
    for (int i = NE - 2; i >= 0; --i) e = e * y + pc[p * PW + i];
    T o = pc[p * PW + NE + NO - 1];
#pragma unroll
    for (int i = NO - 2; i >= 0; --i) o = o * y + pc[p * PW + NE + i];
    w[p] = e + x * o;
    w[TAPS - 1 - p] = e - x * o;
  }
}

// Weight of tap t for a node (general path), offset delta = cK - 1/2 + x/2
// from the node's first tap.  Kaiser-Bessel: the fitted polynomial from the
// instance table, or the kernel itself when no fit met the tolerance.  The
// other methods, scaled like the Kaiser-Bessel weights (which carry
// Psi_hat / 2 against the 1 / (pi c) of the plan's scale):
//   truncated sinc  Psi_hat(u) / 2 = sin(c pi u) / u, u = (delta - t) / c;
//   linear          pi c (1 - |delta - t|);
//   nearest         pi c.
template <typename T>
__device__ __forceinline__ T tap_weight(const Inst& I, int t, T x) {
  if (I.poly) return tap_poly<T>(static_cast<const T*>(I.poly_c) + t * (Deg<T>::v + 1), x);
  const T delta = T(I.ck - 0.5) + T(0.5) * x;
  const T d = delta - T(t);
  switch (I.kind) {
    case 1: {  // truncated sinc: c sin(pi d) / d
      T s, co;
      m_sincospi(d, &s, &co);
      return d == T(0) ? T(kPi * I.c) : T(I.c) * s / d;
    }
    case 2: {
      const T a = d < T(0) ? -d : d;
      return a < T(1) ? T(kPi * I.c) * (T(1) - a) : T(0);
    }
    case 3: return T(kPi * I.c);
    default: return kb_phi<T>(d * T(1.0 / I.c), T(I.K), T(I.alpha));
  }
}

// Node position on the oversampled grid for nu (time-bin units): first tap
// j0 = floor(c nu - cK) + 1 reduced mod m, polynomial offset
// x = 2 (c nu - j0 - cK) + 1 in (-1, 1].
template <typename T>
struct Node {
  int j0;
  T x;
};
template <typename T, bool P2>
__device__ __forceinline__ Node<T> make_node(double nu, const Inst& I, int m, double inv_m) {
  int j00;
  const double d = tap_origin(I.c * nu, I.ck, &j00);
  Node<T> nd;
  nd.x = (T)(2.0 * d + 1.0);
  if constexpr (P2) {
    nd.j0 = j00 & (m - 1);
  } else {
    // j00 mod m without an integer division
    const double j1 = (double)j00;
    int j0 = (int)(j1 - (double)m * floor(j1 * inv_m));
    if (j0 >= m) j0 -= m;
    if (j0 < 0) j0 += m;
    nd.j0 = j0;
  }
  return nd;
}

// sum_t phi((delta - t)/c) U[(j0 + t) mod m] at nu.  With PAIRS the grid line
// carries a halo (U[m + t] = U[t], t < TAPS - 1), so the taps read
// U[j0 .. j0 + TAPS - 1] without wrapping.
template <typename T, int TAPS, bool PAIRS, bool P2, bool HALO = true>
__device__ __forceinline__ cx<T> tap_sum(const cx<T>* U, int m, double inv_m, double nu, const Inst& I,
                                         const StageArgs& a) {
  const Node<T> nd = make_node<T, P2>(nu, I, m, inv_m);
  cx<T> acc = mk(T(0), T(0));
  if constexpr (PAIRS) {
    T w[TAPS];
    tap_weights_pairs<T, TAPS>(a, nd.x, w);
    if (HALO || nd.j0 <= m - TAPS) {
      const cx<T>* u = U + nd.j0;
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
        const cx<T> g = u[t];
        acc.x += w[t] * g.x;
        acc.y += w[t] * g.y;
      }
    } else {
      // the window runs past the end of a line without halo: wrap its taps
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
        int j = nd.j0 + t;
        j -= j >= m ? m : 0;
        const cx<T> g = U[j];
        acc.x += w[t] * g.x;
        acc.y += w[t] * g.y;
      }
    }
  } else {
    int jm = nd.j0;
    for (int t = 0; t < I.taps; ++t) {
      const T w = tap_weight<T>(I, t, nd.x);
      const cx<T> g = U[jm];
      acc.x += w * g.x;
      acc.y += w * g.y;
      if (++jm == m) jm = 0;
    }
  }
  return acc;
}

// a when keep, else b, as a bitwise select (a conditional on array elements
// may be lowered to a select of indices and compare chains)
__device__ __forceinline__ float bitsel(bool keep, float a, float b) {
  const unsigned k = keep ? ~0u : 0u;
  return __uint_as_float((__float_as_uint(a) & k) | (__float_as_uint(b) & ~k));
}
__device__ __forceinline__ double bitsel(bool keep, double a, double b) {
  const unsigned long long k = keep ? ~0ull : 0ull;
  return __longlong_as_double((long long)(((unsigned long long)__double_as_longlong(a) & k) |
                                          ((unsigned long long)__double_as_longlong(b) & ~k)));
}

// j mod m for a first tap j of either sign
template <bool P2>
__device__ __forceinline__ int wrap_tap(int j, int m, double inv_m) {
  if constexpr (P2) {
    return j & (m - 1);
  } else {
    const double jd = (double)j;
    int r = (int)(jd - (double)m * floor(jd * inv_m));
    if (r >= m) r -= m;
    if (r < 0) r += m;
    return r;
  }
}

// sum_t w[t] U[(j + t) mod m], j in [0, m)
template <typename T, int TAPS, bool HALO>
__device__ __forceinline__ cx<T> taps_at(const cx<T>* U, int m, int j, const T* w) {
  cx<T> acc = mk(T(0), T(0));
  if (HALO || j <= m - TAPS) {
    const cx<T>* u = U + j;
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      const cx<T> g = u[t];
      acc.x += w[t] * g.x;
      acc.y += w[t] * g.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      int jt = j + t;
      jt -= jt >= m ? m : 0;
      const cx<T> g = U[jt];
      acc.x += w[t] * g.x;
      acc.y += w[t] * g.y;
    }
  }
  return acc;
}

// The window of a node pair +nup, -nup with the paired taps: the node phase,
// the first taps (reduced mod m) and both nodes' weights.  The two windows
// are mirror images (the kernel is even and cK = TAPS/2 is an integer):
// -nup's first tap is -(j0 + TAPS - 1) and its weights are +nup's reversed,
// except for a node on a grid point (c nup an integer), where both offsets
// are -1: the same weights, first tap -(j0 + TAPS - 2).  So the window
// polynomials run once per pair, and lines with the same nodes share them.
template <typename T, int TAPS>
struct PairWin {
  cx<T> ph;    // exp(-i pi nup) (1 on an uncentred grid)
  int jp, jn;  // first taps of +nup and -nup, in [0, m)
  bool on;     // node on a grid point: -nup takes w itself, not reversed
  T w[TAPS];
};
template <typename T, int TAPS, bool P2>
__device__ __forceinline__ void pair_window(double nup, const Inst& I, const StageArgs& a, int m, double inv_m,
                                            PairWin<T, TAPS>& pw) {
  // (an uncentred grid, the interpolation-based methods, needs no node phase)
  pw.ph = I.centred ? phase_mpi<T>(nup) : mk(T(1), T(0));
  int j0;
  const double d = tap_origin(I.c * nup, I.ck, &j0);
  const T x = (T)(2.0 * d + 1.0);
  const bool ongrid = d == -1.0;
  tap_weights_pairs<T, TAPS>(a, x, pw.w);
  pw.on = ongrid;
  const int jm = ongrid ? -(j0 + TAPS - 2) : -(j0 + TAPS - 1);
  pw.jp = wrap_tap<P2>(j0, m, inv_m);
  pw.jn = wrap_tap<P2>(jm, m, inv_m);
}
// exp(-+i pi nup) sum_t phi(...) U[...] at +nup and -nup on one grid line U
// (m points, with a halo of TAPS - 1 when HALO)
template <typename T, int TAPS, bool HALO>
__device__ __forceinline__ void pair_values(const cx<T>* U, int m, const PairWin<T, TAPS>& pw, cx<T>* vp,
                                            cx<T>* vn) {
  cx<T> sp, sn;
  // the weights of -nup: w reversed, or w itself on a grid point (the
  // reversal costs nothing where no lane of the wave is on one)
  const bool anyon = __any(pw.on);
  auto wm = [&](int t) { return bitsel(pw.on, pw.w[t], pw.w[TAPS - 1 - t]); };
  if (HALO || (pw.jp <= m - TAPS && pw.jn <= m - TAPS)) {
    // both windows in one loop: two independent sums, two reads in flight
    const cx<T>* up = U + pw.jp;
    const cx<T>* un = U + pw.jn;
    sp = sn = mk(T(0), T(0));
    auto sums = [&](auto wmt) {
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
        const cx<T> g = up[t], h = un[t];
        const T b = wmt(t);
        sp.x += pw.w[t] * g.x;
        sp.y += pw.w[t] * g.y;
        sn.x += b * h.x;
        sn.y += b * h.y;
      }
    };
    if (anyon) sums(wm);
    else sums([&](int t) { return pw.w[TAPS - 1 - t]; });
  } else {
    T wms[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) wms[t] = wm(t);
    sp = taps_at<T, TAPS, HALO>(U, m, pw.jp, pw.w);
    sn = taps_at<T, TAPS, HALO>(U, m, pw.jn, wms);
  }
  *vp = cmul(sp, pw.ph);
  *vn = cmul(sn, cconj(pw.ph));
}

// The type-2 values at the node pair +nup and -nup:
// exp(-+i pi nup) sum_t phi(...) U[...]; the two phases are conjugate.  With
// the paired taps by the mirrored windows of pair_window.
template <typename T, int TAPS, bool PAIRS, bool P2, bool HALO = true>
__device__ __forceinline__ void interp_pair(const cx<T>* U, int m, double inv_m, double nup, const Inst& I,
                                            const StageArgs& a, cx<T>* vp, cx<T>* vn) {
  if constexpr (PAIRS) {
    PairWin<T, TAPS> pw;
    pair_window<T, TAPS, P2>(nup, I, a, m, inv_m, pw);
    pair_values<T, TAPS, HALO>(U, m, pw, vp, vn);
  } else {
    const cx<T> ph = I.centred ? phase_mpi<T>(nup) : mk(T(1), T(0));
    *vp = cmul(tap_sum<T, TAPS, PAIRS, P2, HALO>(U, m, inv_m, nup, I, a), ph);
    *vn = cmul(tap_sum<T, TAPS, PAIRS, P2, HALO>(U, m, inv_m, -nup, I, a), cconj(ph));
  }
}

template <bool P2 = false>
__device__ __forceinline__ double line_ak(const Inst& I, int line) {
  int k1, k2i;
  divmod<P2>(line, I.n2, &k1, &k2i);
  const int k2 = 2 * k2i < I.n2 ? k2i : k2i - I.n2;
  return I.a1 * (double)k1 * (double)k1 + I.a2 * (double)k2 * (double)k2;
}

// Lines taken in mirror pairs (3D): line slots 2P and 2P + 1 hold (k1, k2)
// and (k1, -k2) of pair P = k1 (n2/2) + r with k2 = r, r = 1 .. n2/2 - 1,
// and r = 0 gives the lines k2 = 0 and k2 = -n2/2.  The two lines of a pair
// with r > 0 have the same |K_x|, so the same nodes and weights (*shared).
template <bool P2>
__device__ __forceinline__ int mirror_line(const Inst& I, int slot, bool* shared) {
  const int h2 = I.n2 >> 1;
  int k1, r;
  divmod<P2>(slot >> 1, h2, &k1, &r);
  *shared = r != 0;
  const int k2 = (slot & 1) ? (r ? I.n2 - r : h2) : r;
  return k1 * I.n2 + k2;
}

// a3 over a group of nl lines whose grids sit in LDS in natural order at
// U + b*ls, by node pairs: the nodes of l and -l are +nu+ and -nu+ with
// nu+ = sqrt(Ak + b l^2), one lane per pair, sharing nu+, the weight and the
// phase.  mode 0 (R): pairs |l| = 1 .. nz/2; output l gets
// wcoef |l| / nu+ times the value at sign(l) nu+; the Nyquist plane
// l = -nz/2 gets the mean of both, and l = 0 gets 0 (weight 0).  mode 1
// (A^T): pairs |l| = 0 .. nz/2; outputs l and -l both get the mean of the two
// values, no weight.  put(e, value) receives output e = b*nz + l_index.
// akl[b] holds line b's |K_x|^2 term.
template <typename T, int TAPS, bool PAIRS, bool P2, bool HALO = true, typename Ak, typename Put>
__device__ __forceinline__ void interp_lines(const Inst& I, const StageArgs& a, const cx<T>* U, int ls,
                                             Ak akl, int nl, int mode, Put put) {
  const int m = I.m, nz = I.nz, half = nz / 2;
  const double wsc = I.wcoef * I.scale;
  const double inv_m = 1.0 / (double)m;
  const int per = mode == 0 ? half : half + 1;
  for (int e = threadIdx.x; e < nl * per; e += kBlock) {
    int b, p;
    if (mode == 0) {
      divmod<P2>(e, half, &b, &p);
    } else {
      b = e / per;
      p = e - b * per;
    }
    const int la = mode == 0 ? p + 1 : p;
    const double nup = sqrt_nt(akl(b) + I.b * (double)la * (double)la);
    cx<T> vp, vn;
    interp_pair<T, TAPS, PAIRS, P2, HALO>(U + b * ls, m, inv_m, nup, I, a, &vp, &vn);
    const int o = b * nz;
    if (mode == 0) {
      const double w = wsc * (double)la * rcp_nt(nup);
      if (la < half) {
        put(o + la, cscl(vp, T(w)));
        put(o + nz - la, cscl(vn, T(w)));
      } else {
        put(o + half, cscl(cadd(vp, vn), T(0.5 * w)));
        put(o, mk(T(0), T(0)));
      }
    } else {
      const cx<T> v = cscl(cadd(vp, vn), T(0.5 * I.scale));
      put(o + la, v);
      if (la > 0 && la < half) put(o + nz - la, v);
    }
  }
}

// Type-1 spreading of one line, the transpose of interp_lines' sum.  The
// line's nodes are listed in increasing order (the pairs -nu+, +nu+ of each
// |l|), one lane per node: first tap j0 (unreduced), value, and tap weights
// (node-major rows with kPad zeros on
// both sides and an odd stride, so consecutive nodes' rows start on
// different LDS banks).  Cell j then gathers, for each periodic image and
// each tap t, the nodes whose first tap is j - t: a contiguous node range
// whose ends come from the closed form of the node positions, corrected
// against the stored j0 (so the ranges are exact).  Summation is in node
// order: no atomics, deterministic.
//   mode 0 (R^T): nodes -nu+(nz/2 .. 1), +nu+(1 .. nz/2); value
//     conj(W exp(-i pi nu) scale) Qhat_l with l = sign(nu)|l|, except that
//     both Nyquist nodes take Qhat_{-nz/2} with half the weight (l = 0 has
//     weight 0 and is left out).
//   mode 1 (A): nodes -nu+(nz/2 .. 0), +nu+(0 .. nz/2); value
//     (scale / 2) exp(i pi nu) (F_l + F_-l) (single term at l = 0, -nz/2).
// fget(l_index) reads the depth spectrum, put(j, value) receives cell j and
// putk(j, values) the KC cells j .. j + KC - 1 (j a multiple of KC).
// KC = 4 in the stand-alone kernel (16-byte stores); the fused adjoint
// kernel takes KC = 2, whose shorter weight rows keep its LDS within 32 KB.
template <typename T, int KC = 4>
struct SpreadLds {
  // a thread gathers kCells consecutive cells; kPad zeros on both sides of a
  // weight row let it read kCells weights of any node in range without tests
  static constexpr int kCells = KC;
  static constexpr int kPad = kCells - 1;
  static __host__ __device__ constexpr int row(int taps) { return (taps + 2 * kPad) | 1; }
  cx<T>* val;  // [node] value
  T* wts;      // [node][row] tap weights, tap t at kPad + t
  int* j0s;    // [node] first tap, unreduced
  static __device__ __forceinline__ SpreadLds carve(void* base, int nz, int taps) {
    SpreadLds s;
    const int nn = nz + 2;
    s.val = static_cast<cx<T>*>(base);
    s.wts = reinterpret_cast<T*>(s.val + nn);
    s.j0s = reinterpret_cast<int*>(s.wts + nn * row(taps));
    return s;
  }
};

// First tap and weight row of node i at +nup (neg = false) or -nup.  With
// the paired taps the window of -nup is the mirror image of +nup's, as in
// interp_pair (so that spreading stays the exact transpose of interpolation):
// first tap -(j0 + TAPS - 1) with the weights reversed, or -(j0 + TAPS - 2)
// with the same weights for a node on a grid point.
template <typename T, int TAPS, bool PAIRS, int KC>
__device__ __forceinline__ void spread_node(const Inst& I, const StageArgs& a, double nup, bool neg,
                                            SpreadLds<T, KC> L, int i, int taps, int rw) {
  constexpr int P = SpreadLds<T, KC>::kPad;
  T* wi = L.wts + i * rw;
#pragma unroll
  for (int t = 0; t < P; ++t) wi[t] = T(0);
  for (int t = P + taps; t < rw; ++t) wi[t] = T(0);
  if constexpr (PAIRS) {
    int j0;
    const double d = tap_origin(I.c * nup, I.ck, &j0);
    const T x = (T)(2.0 * d + 1.0);
    const bool ongrid = d == -1.0;
    T w[TAPS];
    tap_weights_pairs<T, TAPS>(a, x, w);
    const bool rev = neg && !ongrid;
#pragma unroll
    for (int t = 0; t < TAPS; ++t) wi[P + t] = bitsel(rev, w[TAPS - 1 - t], w[t]);
    L.j0s[i] = !neg ? j0 : (ongrid ? -(j0 + TAPS - 2) : -(j0 + TAPS - 1));
  } else {
    int j0;
    const double d = tap_origin(I.c * (neg ? -nup : nup), I.ck, &j0);
    const T x = (T)(2.0 * d + 1.0);
    L.j0s[i] = j0;
    for (int t = 0; t < taps; ++t) wi[P + t] = tap_weight<T>(I, t, x);
  }
}

template <typename T, int TAPS, bool PAIRS, int KC, typename Fget, typename Put, typename Put4>
__device__ __forceinline__ void spread_line(const Inst& I, const StageArgs& a, int line, int mode, SpreadLds<T, KC> L,
                                            Fget fget, Put put, Put4 put4) {
  const int m = I.m, nz = I.nz, half = nz / 2, taps = PAIRS ? TAPS : I.taps;
  const int q0 = mode == 0 ? 1 : 0;  // smallest |l| listed
  const int nq = half - q0 + 1;      // |l| values, one node pair each
  const int nn = 2 * nq;             // nodes
  const double Ak = line_ak(I, line);
  const double wsc = I.wcoef * I.scale;
  const int rw = SpreadLds<T, KC>::row(taps);
  for (int i = threadIdx.x; i < nn; i += kBlock) {
    // node i: +nu+(q0 + i - nq) for i >= nq, else -nu+(q0 + nq - 1 - i)
    const bool pos = i >= nq;
    const int la = q0 + (pos ? i - nq : nq - 1 - i);
    const double nup = sqrt_nt(Ak + I.b * (double)la * (double)la);
    cx<T> q;
    double cf;
    if (mode == 0) {
      const bool nyq = la == half;
      q = fget(nyq ? half : (pos ? la : nz - la));
      cf = wsc * (double)la * rcp_nt(nup) * (nyq ? 0.5 : 1.0);
    } else {
      q = fget(la);
      if (la != 0 && la != half) q = cadd(q, fget(nz - la));
      cf = 0.5 * I.scale;
    }
    // the value at nu is q conj(exp(-i pi nu)) cf; the phases at +-nup are
    // conjugate
    const cx<T> ph = phase_mpi<T>(nup);
    L.val[i] = cscl(cmul(q, pos ? cconj(ph) : ph), T(cf));
    spread_node<T, TAPS, PAIRS, KC>(I, a, nup, !pos, L, i, taps, rw);
  }
  __syncthreads();
  const int jlo = L.j0s[0];
  const int span = L.j0s[nn - 1] - jlo + 1;
  const double inv_c = 1.0 / I.c, inv_b = 1.0 / I.b;
  // Index of the first node whose first tap is >= jlo + xr.  A node's first
  // tap is below J exactly when nu < X = (J - 1 + cK) / c; the nodes below X
  // are counted from nu+(q)^2 = Ak + b q^2, then the count is moved onto the
  // stored first taps (one or two steps at most in practice).
  auto first_ge = [&](int xr) -> int {
    if (xr <= 0) return 0;
    if (xr >= span) return nn;
    const int J = jlo + xr;
    const double X = ((double)(J - 1) + I.ck) * inv_c;
    const double R = (X * X - Ak) * inv_b;  // bound on q^2
    const double sq = R > 0.0 ? sqrt_nt(R) : 0.0;
    int s;
    if (X > 0.0) {
      // every -nu+ node, then +nu+(q) for q0 <= q < sqrt(R)
      int c = R > 0.0 ? (int)ceil(sq) - q0 : 0;
      c = c < 0 ? 0 : (c > nq ? nq : c);
      s = nq + c;
    } else {
      // -nu+(q) < X  <=>  q^2 > R
      int c = R >= 0.0 ? (int)floor(sq) - q0 + 1 : 0;
      c = c < 0 ? 0 : (c > nq ? nq : c);
      s = nq - c;
    }
    while (s > 0 && L.j0s[s - 1] >= J) --s;
    while (s < nn && L.j0s[s] < J) ++s;
    return s;
  };
  // Each thread owns kCells consecutive cells [j, j + kCells).  For every
  // periodic image (offset v = j + q m - jlo of its first cell, with some
  // cell of the block in [0, span + taps - 1)) the nodes touching the block
  // have first taps in [v - taps + 1, v + kCells - 1]: one contiguous node
  // range.  Node i adds weight (v + c - (j0 - jlo)) times its value to cell
  // c; the padded weight row makes out-of-window taps read zeros.
  constexpr int kCells = SpreadLds<T, KC>::kCells;
  constexpr int P = SpreadLds<T, KC>::kPad;
  const int vend = span + taps - 1;
  for (int j = kCells * (int)threadIdx.x; j < m; j += kCells * kBlock) {
    cx<T> acc[kCells];
#pragma unroll
    for (int c = 0; c < kCells; ++c) acc[c] = mk(T(0), T(0));
    int v = (j - jlo) % m;
    if (v < 0) v += m;
    // the image before may still reach the block's last cells
    if (v - m + kCells - 1 >= 0) v -= m;
    for (; v < vend; v += m) {
      const int i1 = first_ge(v + kCells);
      for (int i = first_ge(v - taps + 1); i < i1; ++i) {
        // taps t0 .. t0 + kCells - 1 with t0 = v - (j0 - jlo) in [-P, taps - 1]
        const T* wr = L.wts + i * rw + (P + v - (L.j0s[i] - jlo));
        const cx<T> vv = L.val[i];
#pragma unroll
        for (int c = 0; c < kCells; ++c) {
          const T w = wr[c];
          acc[c].x += w * vv.x;
          acc[c].y += w * vv.y;
        }
      }
    }
    if (j + kCells <= m) {
      put4(j, acc);
    } else {
#pragma unroll
      for (int c = 0; c < kCells; ++c)
        if (j + c < m) put(j + c, acc[c]);
    }
  }
}

// ---------------------------------------------------------------------------
// Type-1 spreading of a line by one wavefront (FP32), node-parallel.
//
// The gather above runs cell by cell, so a cell where many nodes crowd (near
// the smallest |nu| of a line with large |K_x|, up to ~40 nodes) holds up its
// whole wavefront.  Here every lane owns a node instead and adds its TAPS
// weighted values to cells j0 .. j0 + TAPS - 1, one tap per round.  The node
// list is monotone, so lanes with equal first taps are contiguous; their
// values are summed first (a segmented sum across the lanes, by DPP moves),
// and only the last lane of each such segment adds the sum to its cell.  In a
// round those writers hold distinct first taps, hence distinct cells, and the
// rounds follow each other in program order: no atomics, and the summation
// order is fixed (deterministic).  Every lane does the same work whatever the
// node density: the cost of a crowd is the few extra scan steps of its
// wavefront.

// DPP move of a float across lanes: row_shr:d within rows of 16 lanes, or
// row_bcast:15 / row_bcast:31.  Lanes whose source lies outside the pattern
// read 0 (bound_ctrl); lanes of rows outside ROWS are not written, and every
// use below selects them away.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, ROWS, 0xf, true));
}
// (a double as its two halves)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_mov(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, ROWS, 0xf, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Segments of a key that is monotone over the 64 lanes (equal keys are
// contiguous).  Bit k of `on` is set when the lane adds in step k of the
// segmented inclusive sum: k = 0 .. 3 add lane L - 1, 2, 4, 8 of the same row of
// 16 lanes (Hillis-Steele), k = 4 adds lane 15 of the row before (rows 1 and
// 3), k = 5 adds lane 31 (rows 2 and 3); each only when that lane belongs to
// the lane's own segment.  `use` (wave-uniform) marks the steps any lane
// needs; after them the last lane of a segment (`tail`) holds its sum.
struct WaveSeg {
  unsigned on;
  unsigned use;
  bool tail;
};

__device__ __forceinline__ WaveSeg wave_segments(int key) {
  const int L = (int)(threadIdx.x & 63);
  const int prev = __shfl_up(key, 1, 64);
  const bool head = L == 0 || prev != key;
  const unsigned long long hm = __ballot(head);
  const unsigned long long upto = L == 63 ? ~0ull : ((2ull << L) - 1ull);
  const int ss = 63 - __clzll(hm & upto);  // first lane of the segment
  const int r = L & 15;
  unsigned f = 0;
  f |= (r >= 1 && L - 1 >= ss) ? 1u : 0u;
  f |= (r >= 2 && L - 2 >= ss) ? 2u : 0u;
  f |= (r >= 4 && L - 4 >= ss) ? 4u : 0u;
  f |= (r >= 8 && L - 8 >= ss) ? 8u : 0u;
  f |= (((L >> 4) & 1) && ss <= (L & ~15) - 1) ? 16u : 0u;
  f |= (L >= 32 && ss <= 31) ? 32u : 0u;
  WaveSeg s;
  s.on = f;
  s.tail = L == 63 || ((hm >> (L + 1)) & 1ull);
  unsigned u = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) u |= __ballot((f >> k) & 1u) ? (1u << k) : 0u;
  s.use = __builtin_amdgcn_readfirstlane(u);  // (uniform: keep it in a scalar register)
  return s;
}

template <int BIT, int CTRL, int ROWS = 0xf, typename F>
__device__ __forceinline__ void seg_step(const WaveSeg& s, F& x, F& y) {
  if (s.use & BIT) {
    const F tx = x + dpp_mov<CTRL, ROWS>(x);
    const F ty = y + dpp_mov<CTRL, ROWS>(y);
    const bool on = (s.on & BIT) != 0;
    x = on ? tx : x;
    y = on ? ty : y;
  }
}

template <int BIT, int CTRL, int ROWS = 0xf, typename F>
__device__ __forceinline__ void seg_step2(const WaveSeg& s, F& x, F& y, F& u, F& v) {
  if (s.use & BIT) {
    const F tx = x + dpp_mov<CTRL, ROWS>(x);
    const F ty = y + dpp_mov<CTRL, ROWS>(y);
    const F tu = u + dpp_mov<CTRL, ROWS>(u);
    const F tv = v + dpp_mov<CTRL, ROWS>(v);
    const bool on = (s.on & BIT) != 0;
    x = on ? tx : x;
    y = on ? ty : y;
    u = on ? tu : u;
    v = on ? tv : v;
  }
}

// The same sum over two pairs (x, y) and (u, v) with the same segments.
template <typename F>
__device__ __forceinline__ void seg_sum2(const WaveSeg& s, F& x, F& y, F& u, F& v) {
  seg_step2<1, 0x111>(s, x, y, u, v);
  seg_step2<2, 0x112>(s, x, y, u, v);
  seg_step2<4, 0x114>(s, x, y, u, v);
  seg_step2<8, 0x118>(s, x, y, u, v);
  seg_step2<16, 0x142, 0xa>(s, x, y, u, v);
  seg_step2<32, 0x143, 0xc>(s, x, y, u, v);
}

// Segmented inclusive sum of (x, y) over the lanes (see WaveSeg).
template <typename F>
__device__ __forceinline__ void seg_sum(const WaveSeg& s, F& x, F& y) {
  seg_step<1, 0x111>(s, x, y);         // row_shr:1
  seg_step<2, 0x112>(s, x, y);         // row_shr:2
  seg_step<4, 0x114>(s, x, y);         // row_shr:4
  seg_step<8, 0x118>(s, x, y);         // row_shr:8
  seg_step<16, 0x142, 0xa>(s, x, y);   // row_bcast:15 into rows 1, 3
  seg_step<32, 0x143, 0xc>(s, x, y);   // row_bcast:31 into rows 2, 3
}

// One pass of a wavefront's nodes (monotone first taps j0 over the active
// lanes, which come first): cell (j0 + t) mod m of the LDS line G gains
// w[t] v for t < TAPS.  Inactive lanes carry v = 0 and keys of their own.
// When no writer's window runs past the end of the line, the cells are
// addressed from one base per lane (the tap goes into the instruction's
// offset).  When the active first taps span m cells or more, two segments
// could share a cell modulo m; the writes of each round then go one lane at a
// time.
// The segments of a pass's keys: first taps, with keys of their own for the
// inactive lanes.
__device__ __forceinline__ WaveSeg pass_segments(int j0, bool act) {
  return wave_segments(act ? j0 : (0x40000000 + (int)(threadIdx.x & 63)));
}

template <typename T, int TAPS, bool P2>
__device__ __forceinline__ void spread_pass_wave(cx<T>* G, int m, int j0, bool act, int nact, cx<T> v, const T* w,
                                                 const WaveSeg& sg) {
  const int L = (int)(threadIdx.x & 63);
  const int jf = __shfl(j0, 0, 64), jl = __shfl(j0, nact - 1, 64);
  const bool distinct = (jf > jl ? jf - jl : jl - jf) < m;
  int r;  // j0 mod m
  if constexpr (P2) {
    r = j0 & (m - 1);
  } else {
    r = j0 % m;
    r += r < 0 ? m : 0;
  }
  const bool wr = act && sg.tail;
  const bool flat = distinct && !__any(wr && r > m - TAPS);
  cx<T>* g = G + r;
  auto sum = [&](int t, T& x, T& y) {
    x = w[t] * v.x;
    y = w[t] * v.y;
    seg_sum(sg, x, y);
  };
  if (flat) {
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      T x, y;
      sum(t, x, y);
      if (wr) {
        g[t].x += x;
        g[t].y += y;
      }
      // the next round's reads come after this round's writes
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  } else {
#pragma unroll
    for (int t = 0; t < TAPS; ++t) {
      T x, y;
      sum(t, x, y);
      int c = r + t;
      c -= c >= m ? m : 0;
      if (distinct) {
        if (wr) {
          G[c].x += x;
          G[c].y += y;
        }
      } else {
        for (int k = 0; k < 64; ++k) {
          if (wr && L == k) {
            G[c].x += x;
            G[c].y += y;
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
}

// Both passes of a batch at once, for the common case that spread_line_wave
// checks: no node on a grid point (so the passes share their segments, and
// the weights of -nu+ are those of +nu+ reversed),
// neither pass's writers wrap past the end of the line, and the cells of the
// two passes are disjoint.  Each cell then receives the same terms in the
// same order as in two separate passes, and a round's two read-add-write
// chains overlap.  rp, rm: first taps mod m.
template <typename T, int TAPS>
__device__ __forceinline__ void spread_pair_wave(cx<T>* G, int rp, int rm, bool wr, cx<T> vp, cx<T> vm, const T* w,
                                                 const WaveSeg& sg) {
  cx<T>* gp = G + rp;
  cx<T>* gm = G + rm;
#pragma unroll
  for (int t = 0; t < TAPS; ++t) {
    const T b = w[TAPS - 1 - t];  // -nu+: w reversed (no node on a grid point)
    T xp = w[t] * vp.x, yp = w[t] * vp.y, xm = b * vm.x, ym = b * vm.y;
    seg_sum2(sg, xp, yp, xm, ym);
    if (wr) {
      const cx<T> a = gp[t], b = gm[t];
      gp[t] = mk(a.x + xp, a.y + yp);
      gm[t] = mk(b.x + xm, b.y + ym);
    }
    // the next round's reads come after this round's writes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

// Whether the cells of the two passes of a batch are disjoint modulo m:
// + nodes cover [jf, jl + TAPS - 1] (first taps monotone over the active
// lanes, jf at lane 0, jl at the last), their mirrors at most
// [-(jl + TAPS - 1), -jf + 1]; both spans shorter than m.
template <int TAPS>
__device__ __forceinline__ bool passes_disjoint(int jf, int jl, int m) {
  const int lo_p = jf, len_p = jl + TAPS - jf;
  const int lo_m = -(jl + TAPS - 1), len_m = jl - jf + TAPS + 1;
  if (len_p + len_m > m) return false;
  int d = (lo_m - lo_p) % m;
  d += d < 0 ? m : 0;
  return d >= len_p && d + len_m <= m;
}

// A few nodes (n <= 64 / TAPS, in lanes 0 .. n-1: first tap j0, value v,
// weights w) spread tap-parallel: lane k TAPS + t adds tap t of node k, one
// node per round.
template <typename T, int TAPS, bool P2>
__device__ __forceinline__ void spread_few_wave(cx<T>* G, int m, int n, int j0, cx<T> v, const T* w) {
  const int L = (int)(threadIdx.x & 63);
  const int k = L / TAPS, t = L - k * TAPS;
  const int kk = k < n ? k : 0;
  const int jk = __shfl(j0, kk, 64);
  const T vx = __shfl(v.x, kk, 64), vy = __shfl(v.y, kk, 64);
  T wt = T(0);
#pragma unroll
  for (int i = 0; i < TAPS; ++i) {
    const T wi = __shfl(w[i], kk, 64);
    wt = t == i ? wi : wt;
  }
  int c;
  if constexpr (P2) {
    c = (jk + t) & (m - 1);
  } else {
    c = (jk + t) % m;
    c += c < 0 ? m : 0;
  }
  for (int q = 0; q < n; ++q) {
    if (k == q) {
      G[c].x += wt * vx;
      G[c].y += wt * vy;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

// Spreading of one line by one wavefront into the LDS line G (m cells,
// zeroed here), the same sums as spread_line: lane L of batch k takes
// |l| = q0 + 64k + L and both its nodes +nu+ and -nu+ (one pass each).  The
// two nodes' windows are mirror images: the tap weights of -nu+ are those of
// +nu+ reversed and its first tap is -(j0 + TAPS - 1), except when c nu+ is
// an integer (the node on a grid point), where both nodes' offsets are -1:
// same weights, first tap -(j0 + TAPS - 2).  The grid receives the
// conjugated values, as spread_line's put does.
//   mode 0 (R^T): |l| = 1 .. nz/2, value conj(W exp(-i pi nu) scale) Qhat_l,
//     l = sign(nu)|l|, the Nyquist pair both from Qhat_{-nz/2} at half weight;
//   mode 1 (A): |l| = 0 .. nz/2, value (scale / 2) exp(i pi nu) (F_l + F_-l)
//     (a single term at l = 0 and -nz/2).
// fget(l_index) reads the line's depth spectrum (DFT order).  A batch of at
// most 64 / (2 TAPS) values of |l| (the last one of mode 1) spreads
// tap-parallel.
template <typename T, int TAPS, bool P2, typename Fget>
__device__ __forceinline__ void spread_line_wave(const Inst& I, const StageArgs& a, int line, int mode, int m, int nz,
                                                 cx<T>* G, Fget fget) {
  static_assert(TAPS % 2 == 0, "mirrored windows need an even tap count");
  const int L = (int)(threadIdx.x & 63);
  if constexpr (sizeof(T) == 4) {
    float4* G4 = reinterpret_cast<float4*>(G);
    for (int e = L; e < m / 2; e += 64) G4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    for (int e = L; e < m; e += 64) G[e] = mk(T(0), T(0));
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int half = nz / 2;
  const int q0 = mode == 0 ? 1 : 0;
  const int nq = half - q0 + 1;
  const double Ak = line_ak(I, line);
  const double wsc = I.wcoef * I.scale;
  for (int base = 0; base < nq; base += 64) {
    const int nact = min(64, nq - base);
    const bool act = L < nact;
    const int la = act ? q0 + base + L : q0;
    const double nup = sqrt_nt(Ak + I.b * (double)la * (double)la);
    const cx<T> ph = phase_mpi<T>(nup);
    cx<T> qp, qm;
    double cf;
    if (mode == 0) {
      const bool nyq = la == half;
      qp = fget(nyq ? half : la);
      qm = fget(nyq ? half : nz - la);
      cf = wsc * (double)la * rcp_nt(nup) * (nyq ? 0.5 : 1.0);
    } else {
      cx<T> q = fget(la);
      if (la != 0 && la != half) q = cadd(q, fget(nz - la));
      qp = qm = q;
      cf = 0.5 * I.scale;
    }
    const T cff = act ? (T)cf : T(0);
    const cx<T> vp = cscl(cmul(cconj(qp), ph), cff);
    const cx<T> vm = cscl(cmul(cconj(qm), cconj(ph)), cff);
    // +nu+: first tap j0, offset x, weights w; -nu+ mirrored (see above)
    int j0;
    const double d = tap_origin(I.c * nup, I.ck, &j0);
    const T x = (T)(2.0 * d + 1.0);
    const bool ongrid = d == -1.0;
    T w[TAPS];
    tap_weights_pairs<T, TAPS>(a, x, w);
    // the weights of -nu+ (w reversed, or w on a grid point), formed only on
    // the paths that hold them
    auto mirror_weights = [&](T* wm) {
#pragma unroll
      for (int t = 0; t < TAPS; ++t) wm[t] = bitsel(ongrid, w[t], w[TAPS - 1 - t]);
    };
    const int jm = ongrid ? -(j0 + TAPS - 2) : -(j0 + TAPS - 1);
    if (2 * nact * TAPS <= 64) {
      T wm[TAPS];
      mirror_weights(wm);
      // nodes +nu+ of lanes 0 .. nact-1, then -nu+ of the same lanes
      const int n2 = 2 * nact;
      const int src = L < nact ? L : L - nact;
      const bool neg = L >= nact;
      T ws[TAPS];
#pragma unroll
      for (int t = 0; t < TAPS; ++t) {
        const T a0 = __shfl(w[t], src, 64), a1 = __shfl(wm[t], src, 64);
        ws[t] = neg ? a1 : a0;
      }
      // (every shuffle runs on all lanes, then each lane selects: a shuffle
      // inside one arm of a branch would read lanes the branch left inactive)
      const int jsp = __shfl(j0, src, 64), jsm = __shfl(jm, src, 64);
      const T vpx = __shfl(vp.x, src, 64), vpy = __shfl(vp.y, src, 64);
      const T vmx = __shfl(vm.x, src, 64), vmy = __shfl(vm.y, src, 64);
      const int js = neg ? jsm : jsp;
      cx<T> vs;
      vs.x = neg ? vmx : vpx;
      vs.y = neg ? vmy : vpy;
      spread_few_wave<T, TAPS, P2>(G, m, n2, js, vs, ws);
    } else {
      // equal first taps of +nu+ give equal first taps of -nu+ (and the
      // reverse), so the two passes share their segments unless a node sits
      // on a grid point
      const WaveSeg sg = pass_segments(j0, act);
      const bool anyon = __any(act && ongrid);
      // (lanes 0 and nact - 1 hold the extreme first taps: read them on the
      // scalar unit)
      const int jf = __builtin_amdgcn_readlane(j0, 0), jl = __builtin_amdgcn_readlane(j0, nact - 1);
      int rp, rm;
      if constexpr (P2) {
        rp = j0 & (m - 1);
        rm = jm & (m - 1);
      } else {
        rp = j0 % m;
        rp += rp < 0 ? m : 0;
        rm = jm % m;
        rm += rm < 0 ? m : 0;
      }
      const bool wr = act && sg.tail;
      if (!anyon && passes_disjoint<TAPS>(jf, jl, m) && !__any(wr && (rp > m - TAPS || rm > m - TAPS))) {
        // (no node on a grid point: -nu+ takes w reversed)
        spread_pair_wave<T, TAPS>(G, rp, rm, wr, vp, vm, w, sg);
      } else {
        T wm[TAPS];
        mirror_weights(wm);
        spread_pass_wave<T, TAPS, P2>(G, m, j0, act, nact, vp, w, sg);
        if (anyon) {
          spread_pass_wave<T, TAPS, P2>(G, m, jm, act, nact, vm, wm, pass_segments(jm, act));
        } else {
          spread_pass_wave<T, TAPS, P2>(G, m, jm, act, nact, vm, wm, sg);
        }
      }
    }
  }
}

extern __shared__ __align__(16) unsigned char pat_smem[];

// With a work counter, thread 0 takes the next item and hands it to the
// block through a slot at byte a.item_slot of the dynamic LDS, past every
// buffer of the kernel (the launcher adds it to the request).
__device__ __forceinline__ int next_item(const StageArgs& a, int iter) {
  int item;
  if (a.counter) {
    int* s_item = reinterpret_cast<int*>(pat_smem + a.item_slot);
    __syncthreads();
    if (threadIdx.x == 0) *s_item = (int)atomicAdd(a.counter, 1u);
    __syncthreads();
    item = *s_item;
  } else {
    item = (int)blockIdx.x + iter * (int)gridDim.x;
  }
  return __builtin_amdgcn_readfirstlane(item);
}

__device__ __forceinline__ int find_inst(const StageArgs& a, int item) {
  int i = 0;
  while (i + 1 < a.n && a.off[i + 1] <= item) ++i;
  return i;
}

// Loop over the work items of this workgroup.  I is the item's instance, li
// its index within the instance; new_inst_ is true when the instance differs
// from the previous item's (per-instance LDS tables are then reloaded).
#define PAT_FOR_EACH_ITEM(a)                                              \
  int prev_inst_ = -1;                                                    \
  for (int iter_ = 0;; ++iter_) {                                         \
    const int item_ = next_item(a, iter_);                                \
    if (item_ >= (a).total) break;                                        \
    const int inst_ = __builtin_amdgcn_readfirstlane(find_inst(a, item_)); \
    [[maybe_unused]] const bool new_inst_ = inst_ != prev_inst_;          \
    prev_inst_ = inst_;                                                   \
    const Inst& I = *(a).inst[inst_];                                     \
    const int li = item_ - (a).off[inst_];

#define PAT_END_ITEM \
  __syncthreads();   \
  }

// Two neighbouring complex values (or four reals) as one 16-byte access for
// float; double values are 16 bytes each already.
// NT marks data that no later stage reads back (the operator's input and
// output arrays): it streams past the caches, which keep the intermediate
// arrays that the next stage reads.
template <typename T, bool NT = false>
__device__ __forceinline__ void ld_pair(const cx<T>* p, cx<T>* a, cx<T>* b) {
  if constexpr (sizeof(T) == 4) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f v;
    if constexpr (NT)
      v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    else
      v = *reinterpret_cast<const v4f*>(p);
    *a = mk(v.x, v.y);
    *b = mk(v.z, v.w);
  } else {
    *a = p[0];
    *b = p[1];
  }
}
template <typename T, bool NT = false>
__device__ __forceinline__ void st_pair(cx<T>* p, cx<T> a, cx<T> b) {
  if constexpr (sizeof(T) == 4) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = {a.x, a.y, b.x, b.y};
    if constexpr (NT)
      __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(p));
    else
      *reinterpret_cast<v4f*>(p) = v;
  } else {
    p[0] = a;
    p[1] = b;
  }
}

// Smooth cut-off of the partial-data model (eq. data-part): data sample
// (x1, x2, t) weighs W[b(x1)][b(x2)][b(t)], b(s) = min(s, n - s) clamped to
// E = I.cut_e (the table and its index are described with Inst::cutw).
__device__ __forceinline__ int cut_band(int s, int n, int E) {
  const int d = min(s, n - s);
  return d < E ? d : E;
}

// Copies the cut-off weights of column x2, W[b1][b(x2)][b3] for b1, b3 <= E,
// into ws ((E+1)^2 values in LDS); visible to the block after its next barrier.
template <typename T>
__device__ __forceinline__ void cut_slice(const Inst& I, T* ws, int x2) {
  const int E = I.cut_e, e1 = E + 1;
  const int b2 = I.n2 > 1 ? cut_band(x2, I.n2, E) : E;
  const T* W = static_cast<const T*>(I.cutw);
  for (int e = threadIdx.x; e < e1 * e1; e += kBlock) {
    const int b1 = e / e1, b3 = e - b1 * e1;
    ws[e] = W[(b1 * e1 + b2) * e1 + b3];
  }
}

// Multiplies v, the data samples t and t + 1 of row x1 (real and imaginary
// part), by their cut-off weights from the column's slice ws (b2: the
// column's band); samples at least E from every face keep weight 1.
template <typename T>
__device__ __forceinline__ void cut_pair(const Inst& I, const T* ws, int b2, int x1, int t, int len, cx<T>* v) {
  const int E = I.cut_e;
  const int b1 = cut_band(x1, I.n1, E);
  if (b1 == E && b2 == E && t >= E && t + 1 <= len - E) return;
  const T* w = ws + b1 * (E + 1);
  v->x *= w[cut_band(t, len, E)];
  v->y *= w[cut_band(t + 1, len, E)];
}

// ---------------------------------------------------------------------------
// Transverse passes.  Tiles of consecutive samples (t or z, the contiguous
// axis) by the full transform length; lanes run along the samples, so global
// accesses are contiguous runs.  The real passes pack two neighbouring real
// samples into one complex column (real and imaginary part) and separate the
// two transforms afterwards, so a tile of tb complex columns covers 2 tb
// samples.  Global accesses move two columns (16 bytes in float) per lane
// where the alignment allows it.

template <typename T, int RS>
__global__ __launch_bounds__(kBlock) void k_tr_x1_r2c(StageArgs a) {
  [[maybe_unused]] constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = tw + I.n1;
  if (new_inst_) load_twiddles(tw, I, I.f1);
  const int len = a.len_nz ? I.nz : I.nt;  // even
  const int tb = I.tb;
  const int ntile = (len + 2 * tb - 1) / (2 * tb);
  const int x2 = li / ntile;
  const int t0 = (li - x2 * ntile) * 2 * tb;
  const T* in = static_cast<const T*>(a.in[inst_]);
  cx<T>* out = static_cast<cx<T>*>(a.out[inst_]);
  const int L = I.n1;
  const size_t rstride = (size_t)I.n2 * len;
  const T* in0 = in + (size_t)x2 * len + t0;
  const bool cut = !a.len_nz && I.cut_e;  // data-side pass with a cut-off
  // the column's cut-off weights, read from LDS while the tile is stored
  T* cws = reinterpret_cast<T*>(buf + L * tb);
  const int cb2 = cut && I.n2 > 1 ? cut_band(x2, I.n2, I.cut_e) : I.cut_e;
  if (cut) {
    cut_slice(I, cws, x2);
    __syncthreads();
  }
  if (len % 4 == 0 && tb % 2 == 0) {
    // column pairs: samples t0 + 4c .. t0 + 4c + 3 (len is a multiple of 4)
    const int hb = tb / 2;
    copy_batched<4>(
        L * hb,
        [&](int e) {
          int x, c;
          divmod<true>(e, hb, &x, &c);
          cx<T> u[2] = {mk(T(0), T(0)), mk(T(0), T(0))};
          if (t0 + 4 * c < len)
            ld_pair<T, true>(reinterpret_cast<const cx<T>*>(in0 + x * rstride + 4 * c), &u[0], &u[1]);
          return cx<cx<T>>{u[0], u[1]};
        },
        [&](int e, cx<cx<T>> v) {
          if (cut) {
            int x, c;
            divmod<true>(e, hb, &x, &c);
            if (t0 + 4 * c < len) {
              cut_pair(I, cws, cb2, x, t0 + 4 * c, len, &v.x);
              cut_pair(I, cws, cb2, x, t0 + 4 * c + 2, len, &v.y);
            }
          }
          buf[2 * e] = v.x;
          buf[2 * e + 1] = v.y;
        });
  } else {
    copy_batched<8>(
        L * tb,
        [&](int e) {
          int x, b;
          divmod<true>(e, tb, &x, &b);
          // samples t0 + 2b (real part) and t0 + 2b + 1 (imaginary part); len is even
          return t0 + 2 * b < len ? *reinterpret_cast<const cx<T>*>(in0 + x * rstride + 2 * b) : mk(T(0), T(0));
        },
        [&](int e, cx<T> v) {
          if (cut) {
            int x, b;
            divmod<true>(e, tb, &x, &b);
            if (t0 + 2 * b < len) cut_pair(I, cws, cb2, x, t0 + 2 * b, len, &v);
          }
          buf[e] = v;
        });
  }
  __syncthreads();
  fft_lds<T, RS, false>(buf, I.f1, tw, tb, 1, tb);
  const int32_t* perm = I.perm + I.f1.perm;
  cx<T>* out0 = out + (size_t)x2 * len + t0;
  for (int e = threadIdx.x; e < I.h1 * tb; e += kBlock) {
    int k, b;
    divmod<true>(e, tb, &k, &b);
    if (t0 + 2 * b >= len) continue;
    const int kn = k == 0 ? 0 : L - k;
    const cx<T> z = buf[perm[k] * tb + b];
    const cx<T> zn = cconj(buf[perm[kn] * tb + b]);
    const T h = T(0.5);
    // transforms of the real and imaginary parts
    const cx<T> pa = cscl(cadd(z, zn), h);
    const cx<T> d = csub(z, zn);
    const cx<T> pb = mk(h * d.y, -h * d.x);
    st_pair(out0 + (size_t)k * rstride + 2 * b, pa, pb);
  }
  PAT_END_ITEM
}

template <typename T, int RS>
__global__ __launch_bounds__(kBlock) void k_tr_x2(StageArgs a) {
  [[maybe_unused]] constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = tw + I.n2;
  if (new_inst_) load_twiddles(tw, I, I.f2);
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = I.tb;
  const int ntile = (len + tb - 1) / tb;
  const int k1 = li / ntile;
  const int t0 = (li - k1 * ntile) * tb;
  cx<T>* io = static_cast<cx<T>*>(a.out[inst_]) + (size_t)k1 * I.n2 * len + t0;
  const int L = I.n2;
  const bool inv = a.mode != 0;
  // column pairs b, b + 1 when tb is even (b even; len is even, so both or
  // neither exist), single columns otherwise
  const int hb = tb / 2;
  if (tb % 2 == 0) {
    copy_batched<4>(
        L * hb,
        [&](int e) {
          int x, c;
          divmod<true>(e, hb, &x, &c);
          cx<T> u[2] = {mk(T(0), T(0)), mk(T(0), T(0))};
          if (t0 + 2 * c < len) ld_pair(io + (size_t)x * len + 2 * c, &u[0], &u[1]);
          return cx<cx<T>>{inv ? cconj(u[0]) : u[0], inv ? cconj(u[1]) : u[1]};
        },
        [&](int e, cx<cx<T>> v) {
          buf[2 * e] = v.x;
          buf[2 * e + 1] = v.y;
        });
  } else {
    copy_batched<8>(
        L * tb,
        [&](int e) {
          int x, b;
          divmod<true>(e, tb, &x, &b);
          const cx<T> v = t0 + b < len ? io[(size_t)x * len + b] : mk(T(0), T(0));
          return inv ? cconj(v) : v;
        },
        [&](int e, cx<T> v) { buf[e] = v; });
  }
  __syncthreads();
  fft_lds<T, RS, false>(buf, I.f2, tw, tb, 1, tb);
  const int32_t* perm = I.perm + I.f2.perm;
  if (tb % 2 == 0) {
    for (int e = threadIdx.x; e < L * hb; e += kBlock) {
      int k, c;
      divmod<true>(e, hb, &k, &c);
      if (t0 + 2 * c < len) {
        const cx<T>* s = buf + perm[k] * tb + 2 * c;
        st_pair(io + (size_t)k * len + 2 * c, inv ? cconj(s[0]) : s[0], inv ? cconj(s[1]) : s[1]);
      }
    }
  } else {
    for (int e = threadIdx.x; e < L * tb; e += kBlock) {
      int k, b;
      divmod<true>(e, tb, &k, &b);
      if (t0 + b < len) {
        const cx<T> v = buf[perm[k] * tb + b];
        io[(size_t)k * len + b] = inv ? cconj(v) : v;
      }
    }
  }
  PAT_END_ITEM
}

// k_tr_x1_r2c as a software pipeline (see k_tr_x2_pipe), for one instance,
// len a multiple of 4, tb even and n1 * tb / 2 <= kPipeU * kBlock
// four-sample loads per tile.  With a cut-off on this (data-side) pass, two
// LDS slices of the weight table alternate: the slice of the next tile's
// column is written while the current tile is transformed, and read when
// the next tile is stored into LDS.  LL > 0 fixes the transform length at
// 2^LL (and its FFT stages) at compile time, in all three pipelines.
template <typename T, int RS, int LL = 0>
__global__ __launch_bounds__(kBlock, RS == 0 ? (sizeof(T) == 4 ? 4 : 2) : 1) void k_tr_x1_pipe(StageArgs a);

// k_tr_x2 as a software pipeline for one instance whose tile is at most
// kPipeU column pairs per thread (n2 * tb / 2 <= kPipeU * kBlock, tb even): a
// persistent grid strides over the tiles, and each workgroup issues the
// loads of its next tile into registers right after storing the current one
// into LDS, so they are in flight while the current tile is transformed and
// written back.  The output positions sit in LDS beside the twiddles (a
// table read from memory in the store loop would wait for those loads).
constexpr int kPipeU = 8;
// tile width of the plans (FP32: 16 columns, 8 once a tile of 2^9-point
// columns would pass 64 KB of LDS; FP64: 8, then 4), fixed with the length in
// the instances that take it at compile time
template <typename T>
constexpr int pipe_tb(int ll) { return sizeof(T) == 4 ? (ll >= 9 ? 8 : 16) : (ll >= 9 ? 4 : 8); }
// registers per thread for a prefetched tile of 2^LL points by tb columns
// (LL > 0), or for the largest tile a run-time length may have
template <int LL>
constexpr int pipe_units(int per_col) {
  return LL > 0 ? ((1 << LL) * per_col + kBlock - 1) / kBlock : 0;
}
template <typename T, int RS, int LL = 0>
__global__ __launch_bounds__(kBlock) void k_tr_x2_pipe(StageArgs a) {
  const Inst& I = *a.inst[0];
  const int L = LL > 0 ? 1 << LL : I.n2;
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  int32_t* pos = reinterpret_cast<int32_t*>(tw + L);
  cx<T>* buf = reinterpret_cast<cx<T>*>(pos + ((L + 3) & ~3));
  load_twiddles(tw, I, I.f2);
  const int32_t* perm = I.perm + I.f2.perm;
  for (int e = threadIdx.x; e < L; e += kBlock) pos[e] = perm[e];
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = LL > 0 ? pipe_tb<T>(LL) : I.tb, hb = tb / 2;
  const int ntile = (len + tb - 1) / tb;
  const bool inv = a.mode != 0;
  cx<T>* base = static_cast<cx<T>*>(a.out[0]);
  constexpr int PU = LL > 0 ? pipe_units<LL>(pipe_tb<T>(LL) / 2) : kPipeU;  // column pairs per thread
  cx<T> pre[2 * PU];
  auto fetch = [&](int item) {
    const int k1 = item / ntile;
    const int t0 = (item - k1 * ntile) * tb;
    const cx<T>* io = base + (size_t)k1 * L * len + t0;
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      pre[2 * u] = pre[2 * u + 1] = mk(T(0), T(0));
      if (e < L * hb) {
        int x, c;
        divmod<true>(e, hb, &x, &c);
        if (t0 + 2 * c < len) ld_pair(io + (size_t)x * len + 2 * c, &pre[2 * u], &pre[2 * u + 1]);
      }
    }
  };
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      if (e < L * hb) {
        buf[2 * e] = inv ? cconj(pre[2 * u]) : pre[2 * u];
        buf[2 * e + 1] = inv ? cconj(pre[2 * u + 1]) : pre[2 * u + 1];
      }
    }
    __syncthreads();
    const int k1 = item / ntile;
    const int t0 = (item - k1 * ntile) * tb;
    cx<T>* io = base + (size_t)k1 * L * len + t0;
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    if constexpr (LL > 0) p2_fft<T, (LL > 0 ? LL : 1), false>(buf, tw, tb, 1, tb);
    else fft_lds<T, RS, false>(buf, I.f2, tw, tb, 1, tb);
    for (int e = threadIdx.x; e < L * hb; e += kBlock) {
      int kk, c;
      divmod<true>(e, hb, &kk, &c);
      if (t0 + 2 * c < len) {
        const cx<T>* s = buf + pos[kk] * tb + 2 * c;
        st_pair(io + (size_t)kk * len + 2 * c, inv ? cconj(s[0]) : s[0], inv ? cconj(s[1]) : s[1]);
      }
    }
    __syncthreads();
  }
}

template <typename T, int RS, int LL>
__global__ __launch_bounds__(kBlock, RS == 0 ? (sizeof(T) == 4 ? 4 : 2) : 1) void k_tr_x1_pipe(StageArgs a) {
  [[maybe_unused]] constexpr bool P2 = RS == 0;
  const Inst& I = *a.inst[0];
  const int L = LL > 0 ? 1 << LL : I.n1;
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  int32_t* pos = reinterpret_cast<int32_t*>(tw + L);
  cx<T>* buf = reinterpret_cast<cx<T>*>(pos + ((L + 3) & ~3));
  const bool cut = !a.len_nz && I.cut_e;  // data-side pass with a cut-off
  const int ew = (I.cut_e + 1) * (I.cut_e + 1);
  T* cws0 = reinterpret_cast<T*>(buf + L * I.tb);  // two column slices of the weights
  load_twiddles(tw, I, I.f1);
  const int32_t* perm = I.perm + I.f1.perm;
  for (int e = threadIdx.x; e < L; e += kBlock) pos[e] = perm[e];
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = LL > 0 ? pipe_tb<T>(LL) : I.tb, hb = tb / 2;
  const int ntile = (len + 2 * tb - 1) / (2 * tb);
  const size_t rstride = (size_t)I.n2 * len;
  const T* in = static_cast<const T*>(a.in[0]);
  cx<T>* out = static_cast<cx<T>*>(a.out[0]);
  constexpr int PU = LL > 0 ? pipe_units<LL>(pipe_tb<T>(LL) / 2) : kPipeU;  // column pairs per thread
  cx<T> pre[2 * PU];
  auto fetch = [&](int item) {
    const int x2 = item / ntile;
    const int t0 = (item - x2 * ntile) * 2 * tb;
    const T* in0 = in + (size_t)x2 * len + t0;
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      pre[2 * u] = pre[2 * u + 1] = mk(T(0), T(0));
      if (e < L * hb) {
        int x, c;
        divmod<true>(e, hb, &x, &c);
        if (t0 + 4 * c < len)
          ld_pair<T, true>(reinterpret_cast<const cx<T>*>(in0 + x * rstride + 4 * c), &pre[2 * u], &pre[2 * u + 1]);
      }
    }
  };
  int item = blockIdx.x;
  if (item < a.total) {
    fetch(item);
    if (cut) {
      cut_slice(I, cws0, item / ntile);
      __syncthreads();
    }
  }
  for (int it = 0; item < a.total; item += gridDim.x, ++it) {
    const int x2 = item / ntile;
    const int t0 = (item - x2 * ntile) * 2 * tb;
    const T* cws = cws0 + (it & 1) * ew;
    const int cb2 = cut && I.n2 > 1 ? cut_band(x2, I.n2, I.cut_e) : I.cut_e;
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      if (e < L * hb) {
        cx<T> v0 = pre[2 * u], v1 = pre[2 * u + 1];
        if (cut) {
          int x, c;
          divmod<true>(e, hb, &x, &c);
          if (t0 + 4 * c < len) {
            cut_pair(I, cws, cb2, x, t0 + 4 * c, len, &v0);
            cut_pair(I, cws, cb2, x, t0 + 4 * c + 2, len, &v1);
          }
        }
        buf[2 * e] = v0;
        buf[2 * e + 1] = v1;
      }
    }
    __syncthreads();
    if (item + (int)gridDim.x < a.total) {
      // The next column's weights are loaded before the next tile and
      // written to the other slice after it (last read before the barrier
      // above): their LDS writes then wait for these loads only, not for
      // the tile's.
      const int nx2 = (item + (int)gridDim.x) / ntile;
      T sv[2];
      if (cut) {
        const int e1 = I.cut_e + 1;
        const int b2 = I.n2 > 1 ? cut_band(nx2, I.n2, I.cut_e) : I.cut_e;
        const T* W = static_cast<const T*>(I.cutw);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = (int)threadIdx.x + h * kBlock;
          if (e < ew) {
            const int b1 = e / e1, b3 = e - b1 * e1;
            sv[h] = W[(b1 * e1 + b2) * e1 + b3];
          }
        }
      }
      fetch(item + gridDim.x);
      if (cut) {
        T* dst = cws0 + ((it + 1) & 1) * ew;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int e = (int)threadIdx.x + h * kBlock;
          if (e < ew) dst[e] = sv[h];
        }
      }
    }
    if constexpr (LL > 0) p2_fft<T, (LL > 0 ? LL : 1), false>(buf, tw, tb, 1, tb);
    else fft_lds<T, RS, false>(buf, I.f1, tw, tb, 1, tb);
    cx<T>* out0 = out + (size_t)x2 * len + t0;
    for (int e = threadIdx.x; e < I.h1 * tb; e += kBlock) {
      int kk, b;
      divmod<true>(e, tb, &kk, &b);
      if (t0 + 2 * b >= len) continue;
      const int kn = kk == 0 ? 0 : L - kk;
      const cx<T> z = buf[pos[kk] * tb + b];
      const cx<T> zn = cconj(buf[pos[kn] * tb + b]);
      const T h = T(0.5);
      const cx<T> pa = cscl(cadd(z, zn), h);
      const cx<T> d = csub(z, zn);
      const cx<T> pb = mk(h * d.y, -h * d.x);
      st_pair(out0 + (size_t)kk * rstride + 2 * b, pa, pb);
    }
    __syncthreads();
  }
}

// Inverse DFT over the first axis from bins 0..n1/2 (the others are the
// complex conjugates of their mirror bins), real part.  Two neighbouring
// samples are transformed together: Z = X_a + i X_b inverts to x_a + i x_b.
// The imaginary parts of the bins 0 and n1/2 are dropped, which is what
// taking the real part of the full inverse DFT does.
template <typename T, int RS>
__global__ __launch_bounds__(kBlock) void k_tr_c2r_k1(StageArgs a) {
  [[maybe_unused]] constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = tw + I.n1;
  if (new_inst_) load_twiddles(tw, I, I.f1);
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = I.tb;
  const int ntile = (len + 2 * tb - 1) / (2 * tb);
  const int x2 = li / ntile;
  const int t0 = (li - x2 * ntile) * 2 * tb;
  const cx<T>* in = static_cast<const cx<T>*>(a.in[inst_]);
  T* out = static_cast<T*>(a.out[inst_]);
  const int L = I.n1;
  const int half = L / 2;
  const size_t rstride = (size_t)I.n2 * len;
  const cx<T>* in0 = in + (size_t)x2 * len + t0;
  const bool cut = !a.len_nz && I.cut_e;  // data-side pass with a cut-off
  T* cws = reinterpret_cast<T*>(buf + L * tb);  // the column's cut-off weights
  if (cut) cut_slice(I, cws, x2);
  copy_batched<4>(
      L * tb,
      [&](int e) {
        int k, b;
        divmod<true>(e, tb, &k, &b);
        const int src = k <= half ? k : L - k;
        cx<T> xa = mk(T(0), T(0)), xb = mk(T(0), T(0));
        if (t0 + 2 * b < len) ld_pair(in0 + (size_t)src * rstride + 2 * b, &xa, &xb);
        if (k == 0 || k == half) {
          xa.y = T(0);
          xb.y = T(0);
        } else if (k > half) {
          xa = cconj(xa);
          xb = cconj(xb);
        }
        // Z = xa + i xb, stored conjugated (inverse DFT as conj(FFT(conj(.))))
        return mk(xa.x - xb.y, -(xa.y + xb.x));
      },
      [&](int e, cx<T> v) { buf[e] = v; });
  __syncthreads();
  fft_lds<T, RS, false>(buf, I.f1, tw, tb, 1, tb);
  const int32_t* perm = I.perm + I.f1.perm;
  T* out0 = out + (size_t)x2 * len + t0;
  const int cb2 = cut && I.n2 > 1 ? cut_band(x2, I.n2, I.cut_e) : I.cut_e;
  if (len % 4 == 0 && tb % 2 == 0) {
    // four samples per lane (len is a multiple of 4)
    const int hb = tb / 2;
    for (int e = threadIdx.x; e < L * hb; e += kBlock) {
      int x, c;
      divmod<true>(e, hb, &x, &c);
      if (t0 + 4 * c < len) {
        const cx<T>* y = buf + perm[x] * tb + 2 * c;  // conj of x_a + i x_b
        cx<T> v0 = mk(y[0].x, -y[0].y), v1 = mk(y[1].x, -y[1].y);
        if (cut) {
          cut_pair(I, cws, cb2, x, t0 + 4 * c, len, &v0);
          cut_pair(I, cws, cb2, x, t0 + 4 * c + 2, len, &v1);
        }
        st_pair<T, true>(reinterpret_cast<cx<T>*>(out0 + (size_t)x * rstride + 4 * c), v0, v1);
      }
    }
  } else {
    for (int e = threadIdx.x; e < L * tb; e += kBlock) {
      int x, b;
      divmod<true>(e, tb, &x, &b);
      if (t0 + 2 * b < len) {
        const cx<T> y = buf[perm[x] * tb + b];  // conj of x_a + i x_b
        cx<T> v = mk(y.x, -y.y);
        if (cut) cut_pair(I, cws, cb2, x, t0 + 2 * b, len, &v);
        *reinterpret_cast<cx<T>*>(out0 + (size_t)x * rstride + 2 * b) = v;
      }
    }
  }
  PAT_END_ITEM
}

// k_tr_c2r_k1 as a software pipeline (see k_tr_x2_pipe), for one instance
// without a cut-off on this pass, len a multiple of 4, tb even and
// n1 * tb <= 2 kPipeU * kBlock bins per tile.
template <typename T, int RS, int LL = 0>
__global__ __launch_bounds__(kBlock, RS == 0 ? (sizeof(T) == 4 ? 4 : 2) : 1) void k_tr_c2r_pipe(StageArgs a) {
  const Inst& I = *a.inst[0];
  const int L = LL > 0 ? 1 << LL : I.n1, half = L / 2;
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  int32_t* pos = reinterpret_cast<int32_t*>(tw + L);
  cx<T>* buf = reinterpret_cast<cx<T>*>(pos + ((L + 3) & ~3));
  load_twiddles(tw, I, I.f1);
  const int32_t* perm = I.perm + I.f1.perm;
  for (int e = threadIdx.x; e < L; e += kBlock) pos[e] = perm[e];
  const int len = a.len_nz ? I.nz : I.nt;
  const int tb = LL > 0 ? pipe_tb<T>(LL) : I.tb, hb = tb / 2;
  const int ntile = (len + 2 * tb - 1) / (2 * tb);
  const size_t rstride = (size_t)I.n2 * len;
  const cx<T>* in = static_cast<const cx<T>*>(a.in[0]);
  T* out = static_cast<T*>(a.out[0]);
  constexpr int U = LL > 0 ? pipe_units<LL>(pipe_tb<T>(LL)) : 2 * kPipeU;  // bins per thread
  cx<T> pre[U];
  auto fetch = [&](int item) {
    const int x2 = item / ntile;
    const int t0 = (item - x2 * ntile) * 2 * tb;
    const cx<T>* in0 = in + (size_t)x2 * len + t0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      pre[u] = mk(T(0), T(0));
      if (e < L * tb) {
        int kk, b;
        divmod<true>(e, tb, &kk, &b);
        const int src = kk <= half ? kk : L - kk;
        cx<T> xa = mk(T(0), T(0)), xb = mk(T(0), T(0));
        if (t0 + 2 * b < len) ld_pair(in0 + (size_t)src * rstride + 2 * b, &xa, &xb);
        if (kk == 0 || kk == half) {
          xa.y = T(0);
          xb.y = T(0);
        } else if (kk > half) {
          xa = cconj(xa);
          xb = cconj(xb);
        }
        // Z = xa + i xb, stored conjugated (inverse DFT as conj(FFT(conj(.))))
        pre[u] = mk(xa.x - xb.y, -(xa.y + xb.x));
      }
    }
  };
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = (int)threadIdx.x + u * kBlock;
      if (e < L * tb) buf[e] = pre[u];
    }
    __syncthreads();
    const int x2 = item / ntile;
    const int t0 = (item - x2 * ntile) * 2 * tb;
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    if constexpr (LL > 0) p2_fft<T, (LL > 0 ? LL : 1), false>(buf, tw, tb, 1, tb);
    else fft_lds<T, RS, false>(buf, I.f1, tw, tb, 1, tb);
    T* out0 = out + (size_t)x2 * len + t0;
    for (int e = threadIdx.x; e < L * hb; e += kBlock) {
      int x, c;
      divmod<true>(e, hb, &x, &c);
      if (t0 + 4 * c < len) {
        const cx<T>* y = buf + pos[x] * tb + 2 * c;  // conj of x_a + i x_b
        st_pair<T, true>(reinterpret_cast<cx<T>*>(out0 + (size_t)x * rstride + 4 * c), mk(y[0].x, -y[0].y),
                         mk(y[1].x, -y[1].y));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Line stages: a group of consecutive frequency lines (k1, k2) per work item.

// DFT of length nz along each line, in place.
template <typename T, int RS>
__global__ __launch_bounds__(kBlock) void k_line_fft(StageArgs a) {
  constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  cx<T>* tw = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = tw + I.nz;
  if (new_inst_) load_twiddles(tw, I, I.fz);
  const int L = I.nz;
  const int line0 = li * I.lpw_z;
  const int nl = min(I.lpw_z, I.lines - line0);
  cx<T>* io = static_cast<cx<T>*>(a.out[inst_]) + (size_t)line0 * L;
  const bool inv = a.mode != 0;
  copy_batched<4>(
      nl * L,
      [&](int e) {
        const cx<T> v = io[e];
        return inv ? cconj(v) : v;
      },
      [&](int e, cx<T> v) { buf[e] = v; });
  __syncthreads();
  fft_lds<T, RS, true>(buf, I.fz, tw, nl, L, 1);
  const int32_t* perm = I.perm + I.fz.perm;
  for (int e = threadIdx.x; e < nl * L; e += kBlock) {
    int b, j;
    divmod<P2>(e, L, &b, &j);
    const cx<T> v = buf[b * L + perm[j]];
    io[e] = inv ? cconj(v) : v;
  }
  PAT_END_ITEM
}

// a2 loading: u_n = G_n s_n placed at (n - nt/2) mod m, zeros elsewhere.  The
// centring turns the per-tap factor exp(i pi j / c) of eq. (nufft-a) into a
// shift, leaving only exp(-i pi nu) per node.
template <typename T, bool P2>
__device__ __forceinline__ void load_deconv_pad(const Inst& I, const cx<T>* g, int nl, cx<T>* buf) {
  const int m = I.m, nt = I.nt;
  const T* sn = static_cast<const T*>(I.sn);
  copy_batched<4>(
      nl * m,
      [&](int e) {
        int b, j;
        divmod<P2>(e, m, &b, &j);
        // centred: grid position j holds sample (j + nt/2) mod m; otherwise j
        int n = I.centred ? j + nt / 2 : j;
        if (n >= m) n -= m;
        return n < nt ? cscl(g[(size_t)b * nt + n], sn[n]) : mk(T(0), T(0));
      },
      [&](int e, cx<T> v) { buf[e] = v; });
}

template <typename T, typename G, int RS>
__global__ __launch_bounds__(kBlock) void k_line_a2(StageArgs a) {
  constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  // the twiddle table in LDS before the lines, or read from memory: for
  // long lines, and for power-of-two lengths (their workgroups, one item
  // each, copy the table slower than the FFT reads it from cache; the LDS
  // region stays reserved, which holds the kernel to fewer workgroups per
  // CU: freeing it made the kernel 1.5x slower)
  cx<T>* lds = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = I.twg_m ? lds : lds + I.m;
  const bool twg = P2 || I.twg_m;
  const cx<T>* tw = twg ? static_cast<const cx<T>*>(I.tw) + I.fm.tw : lds;
  if (new_inst_ && !twg) load_twiddles(lds, I, I.fm);
  const int m = I.m, nt = I.nt;
  const int line0 = li * I.lpw_m;
  const int nl = min(I.lpw_m, I.lines - line0);
  load_deconv_pad<T, P2>(I, static_cast<const cx<T>*>(a.in[inst_]) + (size_t)line0 * nt, nl, buf);
  __syncthreads();
  fft_lds<T, RS, true>(buf, I.fm, tw, nl, m, 1);
  const int32_t* perm = I.perm + I.fm.perm;
  G* grid = static_cast<G*>(a.out[inst_]);
  for (int e = threadIdx.x; e < nl * m; e += kBlock) {
    int b, j;
    divmod<P2>(e, m, &b, &j);
    // (power-of-two lengths: the DIF position from the index, no table)
    const int pos = P2 ? dif_position_p2(I.fm, j) : perm[j];
    GridIO<T, G>::st(grid, (size_t)line0 * m + e, buf[b * m + pos]);
  }
  PAT_END_ITEM
}

// Stage a2 alone (the staged and bf16-grid paths) as a software pipeline for
// one FP32 instance with the centred c = 2 grid and m = 2^LM points, the
// first half of k_line_nufft2_pipe_c: a persistent grid strides over line
// groups of 2048/m lines; each workgroup's first FFT stage takes the four
// nonzero samples per butterfly from registers loaded during the previous
// group, the radix plan is compile-time, the last stage writes natural
// order into an LDS buffer, and the grid lines leave it in coalesced stores.
template <typename G, int LM>
__global__ __launch_bounds__(kBlock, 4) void k_line_a2_pipe(StageArgs a) {
  using T = float;
  const Inst& I = *a.inst[0];
  constexpr int m = 1 << LM, nt = m / 2, lpw = 2048 / m;
  using PM = P2Plan<LM, p2_l16_m(LM)>;
  static_assert(PM::rad(0) == 8 && PM::nst >= 2, "pipelined first stage");
  constexpr int PADL = 4;
  auto pad = [](int i) { return i + (i >> PADL); };
  constexpr int sub = m >> 3, lsub = LM - 3;
  const int j = (int)threadIdx.x & (sub - 1), bb = (int)threadIdx.x >> lsub;
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  cx<T>* gn = reinterpret_cast<cx<T>*>(pat_smem);  // grid lines, natural order
  cx<T>* gp = gn + lpw * m;                          // FFT scratch, padded
  const T* sn = static_cast<const T*>(I.sn);
  const int q = nt >> 2;
  // inputs r = 0, 1, 6, 7 of the butterfly: samples j + nt/2, j + 3nt/4, j, j + nt/4
  const int ns[4] = {j + 2 * q, j + 3 * q, j, j + q};
  T snr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) snr[i] = sn[ns[i]];
  const cx<T> w1 = twm[j];
  const cx<T>* in = static_cast<const cx<T>*>(a.in[0]);
  G* grid = static_cast<G*>(a.out[0]);
  cx<T> pre[4];
  auto fetch = [&](int item) {
    const int line = item * lpw + bb;
    const bool ok = line < I.lines;
    const cx<T>* gin = in + (size_t)line * nt;
#pragma unroll
    for (int i = 0; i < 4; ++i) pre[i] = ok ? gin[ns[i]] : mk(T(0), T(0));
  };
  constexpr int step = m / PM::rad(PM::nst - 1);
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
    const int line0 = item * lpw;
    const int nl = min(lpw, I.lines - line0);
    {
      cx<T> v[8];
      v[0] = cscl(pre[0], snr[0]);
      v[1] = cscl(pre[1], snr[1]);
      v[2] = v[3] = v[4] = v[5] = mk(T(0), T(0));
      v[6] = cscl(pre[2], snr[2]);
      v[7] = cscl(pre[3], snr[3]);
      dft_pow2<T, 8>(v);
      twiddle_pow2<T, 8>(v, w1);
#pragma unroll
      for (int r = 0; r < 8; ++r) gp[pad(bb * m + j + r * sub)] = v[r];
    }
    __syncthreads();
    p2_stages<T, LM, 1, p2_l16_m(LM), PADL>(gp, twm, lpw);
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    fft_last_stage_p2<T, PM::rad(PM::nst - 1), true, PADL>(gp, m, lpw, m, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* g = gn + b * m;
      const int k0 = PM::natural(blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) g[k0 + r * step] = v[r];
    });
    __syncthreads();
    for (int e = threadIdx.x; e < nl * m; e += kBlock) GridIO<T, G>::st(grid, (size_t)line0 * m + e, gn[e]);
    __syncthreads();
  }
}

// transpose of a2 on LDS grids (natural order, conjugated on entry by the
// caller): X_n = s_n (inverse DFT of the grid line)[(n - nt/2) mod m]
template <typename T, int RS>
__device__ __forceinline__ void ifft_pick_deconv(const Inst& I, cx<T>* buf, int nl, cx<T>* x, const cx<T>* twm) {
  constexpr bool P2 = RS == 0;
  const int m = I.m, nt = I.nt;
  const T* sn = static_cast<const T*>(I.sn);
  fft_lds<T, RS, true>(buf, I.fm, twm, nl, m, 1);
  const int32_t* perm = I.perm + I.fm.perm;
  for (int e = threadIdx.x; e < nl * nt; e += kBlock) {
    int b, n;
    divmod<P2>(e, nt, &b, &n);
    int k = n - nt / 2;
    if (k < 0) k += m;
    // (power-of-two lengths: the DIF position from the index, no table)
    const int pos = P2 ? dif_position_p2(I.fm, k) : perm[k];
    x[e] = cscl(cconj(buf[b * m + pos]), sn[n]);
  }
}

template <typename T, typename G, int RS>
__global__ __launch_bounds__(kBlock) void k_line_a2t(StageArgs a) {
  constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  // the twiddle table in LDS before the lines, or read from memory (long
  // lines, power-of-two lengths: see k_line_a2)
  cx<T>* lds = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* buf = I.twg_m ? lds : lds + I.m;
  const bool twg = P2 || I.twg_m;
  const cx<T>* tw = twg ? static_cast<const cx<T>*>(I.tw) + I.fm.tw : lds;
  if (new_inst_ && !twg) load_twiddles(lds, I, I.fm);
  const int m = I.m, nt = I.nt;
  const int line0 = li * I.lpw_m;
  const int nl = min(I.lpw_m, I.lines - line0);
  const G* grid = static_cast<const G*>(a.in[inst_]);
  copy_batched<4>(
      nl * m, [&](int e) { return cconj(GridIO<T, G>::ld(grid, (size_t)line0 * m + e)); },
      [&](int e, cx<T> v) { buf[e] = v; });
  __syncthreads();
  ifft_pick_deconv<T, RS>(I, buf, nl, static_cast<cx<T>*>(a.out[inst_]) + (size_t)line0 * nt, tw);
  PAT_END_ITEM
}

// The transpose of a2 alone (the staged paths of R^T and A) as a software
// pipeline for one FP32 instance with the centred c = 2 grid and m = 2^LM
// points: a persistent grid strides over line groups of 2048/m lines; each
// workgroup stores its group's grid lines (conjugated) into a padded LDS
// scratch, issues the loads of the next group into registers, runs the
// compile-time FFT, and its last stage writes the picked, deconvolved time
// samples X_n = s_n conj(G_k), k = (n - nt/2) mod m, straight to memory.
template <typename G, int LM>
__global__ __launch_bounds__(kBlock, 4) void k_line_a2t_pipe(StageArgs a) {
  using T = float;
  const Inst& I = *a.inst[0];
  constexpr int m = 1 << LM, nt = m / 2, lpw = 2048 / m, per = 2048 / kBlock;
  using PM = P2Plan<LM, p2_l16_m(LM)>;
  static_assert(PM::nst >= 2, "two or more stages");
  constexpr int PADL = 4;
  auto pad = [](int i) { return i + (i >> PADL); };
  cx<T>* gp = reinterpret_cast<cx<T>*>(pat_smem);
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const T* sn = static_cast<const T*>(I.sn);
  const G* grid = static_cast<const G*>(a.in[0]);
  cx<T>* xout = static_cast<cx<T>*>(a.out[0]);
  const size_t npts = (size_t)I.lines * m;
  cx<T> pre[per];
  auto fetch = [&](int item) {
    const size_t base = (size_t)item * lpw * m;
#pragma unroll
    for (int u = 0; u < per; ++u) {
      const size_t e = base + threadIdx.x + u * kBlock;
      pre[u] = e < npts ? GridIO<T, G>::ld(grid, e) : mk(T(0), T(0));
    }
  };
  constexpr int step = m / PM::rad(PM::nst - 1);
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
    const int line0 = item * lpw;
    const int nl = min(lpw, I.lines - line0);
#pragma unroll
    for (int u = 0; u < per; ++u) gp[pad((int)threadIdx.x + u * kBlock)] = cconj(pre[u]);
    __syncthreads();
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    p2_stages<T, LM, 0, p2_l16_m(LM), PADL>(gp, twm, lpw);
    fft_last_stage_p2<T, PM::rad(PM::nst - 1), true, PADL>(gp, m, lpw, m, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      if (b >= nl) return;
      const int k0 = PM::natural(blk * R);
      cx<T>* x = xout + (size_t)(line0 + b) * nt;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n = (k0 + r * step + nt / 2) & (m - 1);
        if (n < nt) x[n] = cscl(cconj(v[r]), sn[n]);
      }
    });
    __syncthreads();
  }
}

// Four consecutive grid cells to memory (p 16-byte aligned for the vector
// forms; bf16 falls back to single cells otherwise).
template <typename T, typename G>
__device__ __forceinline__ void grid_store4(G* p, const cx<T>* v) {
  if constexpr (sizeof(G) == 8 && sizeof(T) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
    q[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    q[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
  } else if constexpr (sizeof(G) == 16) {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int c = 0; c < 4; ++c) q[c] = make_double2(v[c].x, v[c].y);
  } else {
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      uint4 u;
      u.x = (uint32_t)f2bf(v[0].x) | ((uint32_t)f2bf(v[0].y) << 16);
      u.y = (uint32_t)f2bf(v[1].x) | ((uint32_t)f2bf(v[1].y) << 16);
      u.z = (uint32_t)f2bf(v[2].x) | ((uint32_t)f2bf(v[2].y) << 16);
      u.w = (uint32_t)f2bf(v[3].x) | ((uint32_t)f2bf(v[3].y) << 16);
      *reinterpret_cast<uint4*>(p) = u;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) GridIO<T, G>::st(p, c, v[c]);
    }
  }
}

// 16-byte chunks of a stored grid line: EPC elements per chunk, unpacked to
// compute precision and stored to LDS (dst is 16-byte aligned).
template <typename T, typename G>
struct GridChunk;
template <>
struct GridChunk<float, cx<float>> {
  static constexpr int EPC = 2;
  static __device__ __forceinline__ void put(uint4 v, cx<float>* dst) { *reinterpret_cast<uint4*>(dst) = v; }
};
template <>
struct GridChunk<double, cx<double>> {
  static constexpr int EPC = 1;
  static __device__ __forceinline__ void put(uint4 v, cx<double>* dst) { *reinterpret_cast<uint4*>(dst) = v; }
};
template <>
struct GridChunk<float, bf2> {
  static constexpr int EPC = 4;
  static __device__ __forceinline__ void put(uint4 v, cx<float>* dst) {
    float4 lo, hi;
    lo.x = __uint_as_float(v.x << 16);
    lo.y = __uint_as_float(v.x & 0xffff0000u);
    lo.z = __uint_as_float(v.y << 16);
    lo.w = __uint_as_float(v.y & 0xffff0000u);
    hi.x = __uint_as_float(v.z << 16);
    hi.y = __uint_as_float(v.z & 0xffff0000u);
    hi.z = __uint_as_float(v.w << 16);
    hi.w = __uint_as_float(v.w & 0xffff0000u);
    reinterpret_cast<float4*>(dst)[0] = lo;
    reinterpret_cast<float4*>(dst)[1] = hi;
  }
};

// a3 alone on the stored grid of one instance, streamed.  A persistent
// workgroup walks line groups (lpw_i lines) with stride gridDim.x; the next
// group's grid is loaded into registers (16-byte loads) before the current
// group is interpolated, so each workgroup keeps its memory requests in
// flight while it computes.  One LDS buffer of lpw_i lines (with a halo of
// TAPS - 1 and a stride rounded to 16 bytes), refilled after a barrier that
// follows the interpolation: half the LDS of a double buffer, so one more
// workgroup fits a compute unit, which is worth the extra barrier.
template <typename T, typename G, int TAPS, bool P2, int NPRE>
__global__ __launch_bounds__(kBlock) void k_line_interp_stream(StageArgs a) {
  using C = GridChunk<T, G>;
  constexpr int EPC = C::EPC;
  constexpr int H = TAPS - 1;
  constexpr int Q = 16 / (int)sizeof(cx<T>) > 0 ? 16 / (int)sizeof(cx<T>) : 1;
  const Inst& I = *a.inst[0];
  const int m = I.m, nz = I.nz, lpw = I.lpw_i, lines = I.lines;
  const int ls = (m + H + Q - 1) / Q * Q;
  const int ngroups = a.total;
  const G* grid = static_cast<const G*>(a.in[0]);
  cx<T>* out = static_cast<cx<T>*>(a.out[0]);
  cx<T>* bufs = reinterpret_cast<cx<T>*>(pat_smem);
  __shared__ double s_ak[2][16];
  uint4 pre[NPRE];
  auto fetch = [&](int g) {
    const int line0 = g * lpw;
    const int nch = min(lpw, lines - line0) * m / EPC;
    const uint4* src = reinterpret_cast<const uint4*>(grid + (size_t)line0 * m);
#pragma unroll
    for (int u = 0; u < NPRE; ++u) {
      const int c = (int)threadIdx.x + u * kBlock;
      if (c < nch) pre[u] = src[c];
    }
  };
  int g = blockIdx.x;
  if (g >= ngroups) return;
  fetch(g);
  for (int k = 0; g < ngroups; g += gridDim.x, ++k) {
    cx<T>* buf = bufs;
    const int line0 = g * lpw;
    const int nl = min(lpw, lines - line0);
    const int nch = nl * m / EPC;
#pragma unroll
    for (int u = 0; u < NPRE; ++u) {
      const int c = (int)threadIdx.x + u * kBlock;
      if (c < nch) {
        int b, j;
        divmod<P2>(c * EPC, m, &b, &j);
        cx<T>* dst = buf + b * ls + j;
        C::put(pre[u], dst);
        if (j < H) {
#pragma unroll
          for (int e = 0; e < EPC; ++e)
            if (j + e < H) dst[m + e] = dst[e];
        }
      }
    }
    if ((int)threadIdx.x < nl) s_ak[k & 1][threadIdx.x] = line_ak(I, line0 + (int)threadIdx.x);
    if (g + (int)gridDim.x < ngroups) fetch(g + (int)gridDim.x);
    __syncthreads();
    cx<T>* o = out + (size_t)line0 * nz;
    const double* akk = s_ak[k & 1];
    interp_lines<T, TAPS, true, P2>(I, a, buf, ls, [&](int b) { return akk[b]; }, nl, a.mode,
                                    [&](int e, cx<T> v) { o[e] = v; });
    __syncthreads();  // every read of the buffer is done before it is refilled
  }
}

// a3 alone: grid lines from memory, weighted node values to memory.
template <typename T, typename G, int TAPS, bool P2>
__global__ __launch_bounds__(kBlock) void k_line_interp(StageArgs a) {
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  __shared__ double s_ak[16];
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nz = I.nz;
  const int line0 = li * I.lpw_i;
  const int nl = min(I.lpw_i, I.lines - line0);
  const bool pairs = TAPS > 0 && a.pair_ok;
  const int H = pairs ? TAPS - 1 : 0;
  const int ls = m + H;
  const G* grid = static_cast<const G*>(a.in[inst_]);
  copy_batched<4>(
      nl * m, [&](int e) { return GridIO<T, G>::ld(grid, (size_t)line0 * m + e); },
      [&](int e, cx<T> v) {
        const int b = e / m;
        const int j = e - b * m;
        buf[b * ls + j] = v;
        if (j < H) buf[b * ls + m + j] = v;
      });
  if (threadIdx.x < nl) s_ak[threadIdx.x] = line_ak(I, line0 + threadIdx.x);
  __syncthreads();
  cx<T>* out = static_cast<cx<T>*>(a.out[inst_]) + (size_t)line0 * nz;
  if (pairs) {
    interp_lines<T, (TAPS > 0 ? TAPS : 2), true, P2>(I, a, buf, ls, [&](int b) { return s_ak[b]; }, nl, a.mode,
                                                     [&](int e, cx<T> v) { out[e] = v; });
  } else {
    interp_lines<T, 0, false, P2>(I, a, buf, ls, [&](int b) { return s_ak[b]; }, nl, a.mode,
                                  [&](int e, cx<T> v) { out[e] = v; });
  }
  PAT_END_ITEM
}

// spreading alone: depth spectra from memory, grid lines to memory.
template <typename T, typename G, int TAPS>
__global__ __launch_bounds__(kBlock) void k_line_spread(StageArgs a) {
  PAT_FOR_EACH_ITEM(a)
  const SpreadLds<T> L = SpreadLds<T>::carve(pat_smem, I.nz, I.taps);
  const cx<T>* F = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)li * I.nz;
  G* grid = static_cast<G*>(a.out[inst_]);
  const size_t row = (size_t)li * I.m;
  auto fget = [&](int l) { return F[l]; };
  auto put = [&](int j, cx<T> v) { GridIO<T, G>::st(grid, row + j, v); };
  auto put4 = [&](int j, const cx<T>* v) { grid_store4<T, G>(grid + row + j, v); };
  if (TAPS > 0 && a.pair_ok) {
    spread_line<T, (TAPS > 0 ? TAPS : 2), true>(I, a, li, a.mode, L, fget, put, put4);
  } else {
    spread_line<T, 0, false>(I, a, li, a.mode, L, fget, put, put4);
  }
  PAT_END_ITEM
}

// Fused a2 + a3 + inverse depth DFT (operators R and A^T): per group of nl
// lines, the detector spectrum is deconvolved, padded and transformed in
// LDS, brought to natural order, interpolated at the line's nodes, and the
// node values are inverse-transformed over depth before the only store.
template <typename T, int RS, int TAPS>
__global__ __launch_bounds__(kBlock) void k_line_nufft2(StageArgs a) {
  constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nt = I.nt, nz = I.nz;
  const int lpw = I.lpw_f;
  const int line0 = li * lpw;
  const int nl = min(lpw, I.lines - line0);
  const bool pairs = TAPS > 0 && a.pair_ok;
  // (no halo: the rare windows that run past the end of a line wrap their
  // taps, which keeps two lines' buffers within 32 KB of LDS)
  const int ls = m;
  auto ak = [&](int b) { return line_ak(I, line0 + b); };
  const int sp = m > nz ? m : nz;
  // (twiddles stay in global memory here: an LDS copy costs this kernel a
  // resident workgroup per CU and the strided reads conflict on banks)
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  cx<T>* gp = reinterpret_cast<cx<T>*>(pat_smem);  // FFT output (permuted order), later the depth line
  cx<T>* gn = gp + lpw * sp;                         // grid in natural order, with halo
  const cx<T>* gin = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)line0 * nt;
  if constexpr (P2) {
    // the first FFT stage reads the deconvolved, centred samples from memory
    // (grid position j holds sample (j + nt/2) mod m, zero from nt on); the
    // last writes the grid in natural order (with its halo)
    const T* sn = static_cast<const T*>(I.sn);
    auto src = [&](int b, int j) {
      int n = j + nt / 2;
      if (n >= m) n -= m;
      return n < nt ? cscl(gin[(size_t)b * nt + n], sn[n]) : mk(T(0), T(0));
    };
    const int step = m / I.fm.rad[I.fm.nst - 1];  // weight of the last digit in k
    fft_lds_p2_src_sink<T, true>(gp, I.fm, twm, nl, m, 1, src, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* g = gn + b * ls;
      const int k0 = dif_natural_p2(I.fm, blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) g[k0 + r * step] = v[r];
    });
  } else {
    load_deconv_pad<T, P2>(I, gin, nl, gp);
    __syncthreads();
    fft_lds<T, RS, true>(gp, I.fm, twm, nl, m, 1);
    const int32_t* permm = I.perm + I.fm.perm;
    for (int e = threadIdx.x; e < nl * m; e += kBlock) {
      int b, j;
      divmod<P2>(e, m, &b, &j);
      gn[b * ls + j] = gp[b * m + permm[j]];
    }
    __syncthreads();
  }
  cx<T>* fz = gp;  // the permuted grid is no longer needed
  if (pairs) {
    interp_lines<T, (TAPS > 0 ? TAPS : 2), true, P2, false>(I, a, gn, ls, ak, nl, a.mode,
                                                            [&](int e, cx<T> v) { fz[e] = cconj(v); });
  } else {
    interp_lines<T, 0, false, P2>(I, a, gn, ls, ak, nl, a.mode, [&](int e, cx<T> v) { fz[e] = cconj(v); });
  }
  __syncthreads();
  cx<T>* out = static_cast<cx<T>*>(a.out[inst_]) + (size_t)line0 * nz;
  if constexpr (P2) {
    // the last stage stores each output at its natural position: for a given
    // r, a wave's butterflies cover one contiguous run of the line
    const int stepz = nz / I.fz.rad[I.fz.nst - 1];
    fft_lds_p2_sink<T, true>(fz, I.fz, twz, nl, nz, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* o = out + b * nz;
      const int k0 = dif_natural_p2(I.fz, blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) o[k0 + r * stepz] = cconj(v[r]);
    });
  } else {
    fft_lds<T, RS, true>(fz, I.fz, twz, nl, nz, 1);
    const int32_t* permz = I.perm + I.fz.perm;
    for (int e = threadIdx.x; e < nl * nz; e += kBlock) {
      int b, j;
      divmod<P2>(e, nz, &b, &j);
      out[e] = cconj(fz[b * nz + permz[j]]);
    }
  }
  PAT_END_ITEM
}

// k_line_nufft2 as a software pipeline for one FP32 instance with c = 2
// (m = 2 nt), power-of-two lengths, a first radix of 8 and exactly one
// first-stage butterfly per thread ((m / 8) lpw_f = kBlock).  With c = 2 and
// the centred padding, butterfly j of a line takes the samples j, j + nt/4,
// j + nt/2 and j + 3nt/4 (the other four inputs are zeros).  A persistent grid
// strides over the line groups; each workgroup loads its next group's
// samples into registers before the last stage of the oversampled FFT, so
// they are in flight through that stage and the interpolation, which load
// nothing else from memory.  The deconvolution factors and the first-stage
// twiddle of a thread are the same for every group and are read once.
template <typename T, int TAPS>
__global__ __launch_bounds__(kBlock, 5) void k_line_nufft2_pipe(StageArgs a) {
  const Inst& I = *a.inst[0];
  const int m = I.m, nt = I.nt, nz = I.nz, lpw = I.lpw_f;
  const int sub = m >> 3, lsub = __builtin_ctz((unsigned)sub);
  const int j = (int)threadIdx.x & (sub - 1), bb = (int)threadIdx.x >> lsub;
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  cx<T>* gp = reinterpret_cast<cx<T>*>(pat_smem);  // FFT scratch, later the depth lines
  cx<T>* gn = gp + lpw * m;                          // grid lines in natural order
  const T* sn = static_cast<const T*>(I.sn);
  const int q = nt >> 2;
  // inputs r = 0, 1, 6, 7 of the butterfly: samples j + nt/2, j + 3nt/4, j, j + nt/4
  const int ns[4] = {j + 2 * q, j + 3 * q, j, j + q};
  T snr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) snr[i] = sn[ns[i]];
  const cx<T> w1 = twm[j];
  const cx<T>* in = static_cast<const cx<T>*>(a.in[0]);
  cx<T>* outb = static_cast<cx<T>*>(a.out[0]);
  cx<T> pre[4];
  auto fetch = [&](int item) {
    const int line0 = item * lpw;
    const bool ok = line0 + bb < I.lines;
    const cx<T>* gin = in + (size_t)(line0 + bb) * nt;
#pragma unroll
    for (int i = 0; i < 4; ++i) pre[i] = ok ? gin[ns[i]] : mk(T(0), T(0));
  };
  const int step = m / I.fm.rad[I.fm.nst - 1];
  const int stepz = nz / I.fz.rad[I.fz.nst - 1];
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
    const int line0 = item * lpw;
    const int nl = min(lpw, I.lines - line0);
    {
      cx<T> v[8];
      v[0] = cscl(pre[0], snr[0]);
      v[1] = cscl(pre[1], snr[1]);
      v[2] = v[3] = v[4] = v[5] = mk(T(0), T(0));
      v[6] = cscl(pre[2], snr[2]);
      v[7] = cscl(pre[3], snr[3]);
      dft_pow2<T, 8>(v);
      twiddle_pow2<T, 8>(v, w1);
      cx<T>* p = gp + bb * m + j;
#pragma unroll
      for (int r = 0; r < 8; ++r) p[r * sub] = v[r];
    }
    __syncthreads();
    int Li = sub;
    for (int s = 1; s + 1 < I.fm.nst; ++s) {
      const int R = I.fm.rad[s];
      if (R == 8) fft_stage<T, 8, true, true>(gp, Li, m, twm, lpw, m, 1);
      else if (R == 4) fft_stage<T, 4, true, true>(gp, Li, m, twm, lpw, m, 1);
      else fft_stage<T, 2, true, true>(gp, Li, m, twm, lpw, m, 1);
      __syncthreads();
      Li /= R;
    }
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    auto sink = [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* g = gn + b * m;
      const int k0 = dif_natural_p2(I.fm, blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) g[k0 + r * step] = v[r];
    };
    {
      const int R = I.fm.rad[I.fm.nst - 1];
      if (R == 8) fft_last_stage_p2<T, 8, true>(gp, m, lpw, m, 1, sink);
      else if (R == 4) fft_last_stage_p2<T, 4, true>(gp, m, lpw, m, 1, sink);
      else fft_last_stage_p2<T, 2, true>(gp, m, lpw, m, 1, sink);
    }
    __syncthreads();
    cx<T>* fz = gp;
    interp_lines<T, TAPS, true, true, false>(I, a, gn, m, [&](int b) { return line_ak(I, line0 + b); }, nl, a.mode,
                                             [&](int e, cx<T> v) { fz[e] = cconj(v); });
    __syncthreads();
    cx<T>* out = outb + (size_t)line0 * nz;
    fft_lds_p2_sink<T, true>(fz, I.fz, twz, nl, nz, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* o = out + b * nz;
      const int k0 = dif_natural_p2(I.fz, blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) o[k0 + r * stepz] = cconj(v[r]);
    });
  }
}

// k_line_nufft2_pipe for m = 2^LM and nz = 2^LZ known at compile time (the
// line group then holds 2^(11 - LM) lines): the same work, with the FFT
// stages, their loops and the output positions fixed by P2Plan.  Bounded at
// four waves per SIMD (128 registers): a five-wave cap (96) made several
// instances spill, while those that need no more than 96 still run five.
// In FP64 (twice the registers and LDS) at two.
template <typename T, int TAPS, int LM, int LZ>
__global__ __launch_bounds__(kBlock, sizeof(T) == 4 ? 4 : 2) void k_line_nufft2_pipe_c(StageArgs a) {
  const Inst& I = *a.inst[0];
  constexpr int m = 1 << LM, nt = m / 2, nz = 1 << LZ, lpw = 2048 / m;
  using PM = P2Plan<LM, p2_l16_m(LM)>;
  using PZ = P2Plan<LZ, p2_l16_z(LZ)>;
  static_assert(PM::rad(0) == 8 && PM::nst >= 2 && LZ <= LM, "pipelined first stage");
  const int sub = m >> 3, lsub = __builtin_ctz((unsigned)sub);
  const int j = (int)threadIdx.x & (sub - 1), bb = (int)threadIdx.x >> lsub;
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  // grid lines in natural order at the start of LDS (the tap reads then take
  // their offsets as immediates), then the FFT scratch (later the depth
  // lines), padded by one point every 16: its strided stages spread over the
  // LDS banks
  constexpr int PADL = 4;
  auto pad = [](int i) { return i + (i >> PADL); };
  cx<T>* gn = reinterpret_cast<cx<T>*>(pat_smem);
  cx<T>* gp = gn + lpw * m;
  const T* sn = static_cast<const T*>(I.sn);
  const int q = nt >> 2;
  // inputs r = 0, 1, 6, 7 of the butterfly: samples j + nt/2, j + 3nt/4, j, j + nt/4
  const int ns[4] = {j + 2 * q, j + 3 * q, j, j + q};
  T snr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) snr[i] = sn[ns[i]];
  const cx<T> w1 = twm[j];
  const cx<T>* in = static_cast<const cx<T>*>(a.in[0]);
  cx<T>* outb = static_cast<cx<T>*>(a.out[0]);
  cx<T> pre[4];
  auto fetch = [&](int item) {
    const int line0 = item * lpw;
    const bool ok = line0 + bb < I.lines;
    const cx<T>* gin = in + (size_t)(line0 + bb) * nt;
#pragma unroll
    for (int i = 0; i < 4; ++i) pre[i] = ok ? gin[ns[i]] : mk(T(0), T(0));
  };
  constexpr int step = m / PM::rad(PM::nst - 1);
  constexpr int stepz = nz / PZ::rad(PZ::nst - 1);
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
    const int line0 = item * lpw;
    const int nl = min(lpw, I.lines - line0);
    {
      cx<T> v[8];
      v[0] = cscl(pre[0], snr[0]);
      v[1] = cscl(pre[1], snr[1]);
      v[2] = v[3] = v[4] = v[5] = mk(T(0), T(0));
      v[6] = cscl(pre[2], snr[2]);
      v[7] = cscl(pre[3], snr[3]);
      dft_pow2<T, 8>(v);
      twiddle_pow2<T, 8>(v, w1);
#pragma unroll
      for (int r = 0; r < 8; ++r) gp[pad(bb * m + j + r * sub)] = v[r];
    }
    __syncthreads();
    p2_stages<T, LM, 1, p2_l16_m(LM), PADL>(gp, twm, lpw);
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    auto sink = [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      cx<T>* g = gn + b * m;
      const int k0 = PM::natural(blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) g[k0 + r * step] = v[r];
    };
    fft_last_stage_p2<T, PM::rad(PM::nst - 1), true, PADL>(gp, m, lpw, m, 1, sink);
    __syncthreads();
    cx<T>* fz = gp;
    interp_lines<T, TAPS, true, true, false>(I, a, gn, m, [&](int b) { return line_ak<true>(I, line0 + b); }, nl, a.mode,
                                             [&](int e, cx<T> v) { fz[pad(e)] = cconj(v); });
    __syncthreads();
    cx<T>* out = outb + (size_t)line0 * nz;
    p2_stages<T, LZ, 0, p2_l16_z(LZ), PADL>(fz, twz, lpw);
    fft_last_stage_p2<T, PZ::rad(PZ::nst - 1), true, PADL>(fz, nz, lpw, nz, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      if (b >= nl) return;
      cx<T>* o = out + b * nz;
      const int k0 = PZ::natural(blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) o[k0 + r * stepz] = cconj(v[r]);
    });
    __syncthreads();
  }
}

// Entries k < L / r of the twiddle table that the twiddled stages (all but
// the last) of a compile-time plan read, r the smallest of their radices.
template <typename Pl, int L>
constexpr int twiddle_extent() {
  int r = 16;
  for (int s = 0; s + 1 < Pl::nst; ++s) r = Pl::rad(s) < r ? Pl::rad(s) : r;
  return L / r;
}
// Waves per SIMD of k_line_nufft2_mirror: four in FP32, two in FP64 (its
// registers).
template <typename T>
constexpr int mirror_waves() { return sizeof(T) == 4 ? 4 : 2; }
// LDS of k_line_nufft2_mirror with NT threads: its 16 NT padded points, the
// twiddles of both FFTs' twiddled stages and, where the workgroups of
// mirror_waves per SIMD still fit in 160 KB, the deconvolution factors s_n.
template <typename T, int LM, int NT>
struct MirrorLds {
  static constexpr int m = 1 << LM, nt = m / 2, nz = m / 4, P = 16 * NT, cs = 2 * (int)sizeof(T);
  static constexpr int TWM = twiddle_extent<P2Plan<LM, p2_l16_m(LM)>, m>();
  static constexpr int TWZ = twiddle_extent<P2Plan<LM - 2, p2_l16_z(LM - 2)>, nz>();
  static constexpr int kPts = P + (P >> 4);
  static constexpr int kTw = (TWM + TWZ) * cs, kSn = nt * (int)sizeof(T);
  static constexpr int kGroups = 4 * mirror_waves<T>() * 64 / NT;  // workgroups per CU
  static constexpr bool SN = (kPts * cs + kTw + kSn) * kGroups <= 160 * 1024;
  static constexpr int bytes = kPts * cs + kTw + (SN ? kSn : 0);
  static constexpr bool fits = bytes * kGroups <= 160 * 1024;
};
static_assert(MirrorLds<float, 10, 256>::TWM == 128 && MirrorLds<float, 10, 256>::TWZ == 64 &&
                  MirrorLds<float, 10, 256>::SN && !MirrorLds<float, 11, 256>::SN &&
                  MirrorLds<float, 11, 256>::fits && MirrorLds<float, 10, 128>::fits &&
                  MirrorLds<double, 10, 128>::fits && MirrorLds<double, 11, 256>::fits,
              "the resident waves per SIMD fit in LDS");

// k_line_nufft2_pipe_c for R on 3D plans whose depth lines are a quarter of
// the grid lines (nz = m/4, m = 2^LM), with NT threads: a work item holds
// NL = 16 NT/m lines, taken in mirror pairs (mirror_line), in 16 NT padded
// points of LDS (four waves per SIMD in FP32, two in FP64).  Each thread runs
// two first-stage butterflies, and in the interpolation one node pair of one
// mirror pair: its window, phase and weight serve both lines (the two lines
// of a pair with r = 0 form their own).  The last grid-FFT stage works in
// place: every thread reads its butterflies' 16 points, and after a barrier
// writes them in natural order over the scratch; the interpolation outputs
// wait in registers for a barrier and then overwrite the grid as the depth
// lines.
template <typename T, int TAPS, int LM, int LZ, int NT>
__global__ __launch_bounds__(NT, mirror_waves<T>()) void k_line_nufft2_mirror(StageArgs a) {
  const Inst& I = *a.inst[0];
  constexpr int m = 1 << LM, nt = m / 2, nz = 1 << LZ, NL = 16 * NT / m, half = nz / 2;
  using PM = P2Plan<LM, p2_l16_m(LM)>;
  using PZ = P2Plan<LZ, p2_l16_z(LZ)>;
  static_assert(LZ == LM - 2 && NL >= 2 && (NL / 2) * half == NT, "one node pair of one mirror pair per thread");
  static_assert(PM::rad(0) == 8 && PM::nst >= 2, "pipelined first stage");
  constexpr int PADL = 4;
  constexpr int LS = m + (m >> PADL);  // line stride in LDS
  auto pad = [](int i) { return i + (i >> PADL); };
  constexpr int sub = m >> 3, lsub = LM - 3;
  constexpr int LPP = NT / sub;  // lines of one pass of first-stage butterflies (NL / 2)
  const int j = (int)threadIdx.x & (sub - 1), bb = (int)threadIdx.x >> lsub;
  using ML = MirrorLds<T, LM, NT>;
  cx<T>* buf = reinterpret_cast<cx<T>*>(pat_smem);
  // the item-invariant tables, copied once into LDS after the points (read
  // at every item, they would otherwise wait on the L2 there)
  cx<T>* twm = buf + ML::kPts;
  cx<T>* twz = twm + ML::TWM;
  T* snl = reinterpret_cast<T*>(twz + ML::TWZ);
  {
    const cx<T>* gm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
    const cx<T>* gz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
    for (int i = threadIdx.x; i < ML::TWM; i += NT) twm[i] = gm[i];
    for (int i = threadIdx.x; i < ML::TWZ; i += NT) twz[i] = gz[i];
    if constexpr (ML::SN) {
      const T* gs = static_cast<const T*>(I.sn);
      for (int i = threadIdx.x; i < nt; i += NT) snl[i] = gs[i];
    }
    __syncthreads();
  }
  auto sn_at = [&](int n) {
    if constexpr (ML::SN) return snl[n];
    return static_cast<const T*>(I.sn)[n];
  };
  const int q = nt >> 2;
  // inputs r = 0, 1, 6, 7 of a butterfly: samples j + nt/2, j + 3nt/4, j, j + nt/4
  // (formed where used: nothing per thread is held across the item loop that
  // can be recomputed)
  auto ns = [&](int i) { return j + (i == 0 ? 2 * q : i == 1 ? 3 * q : i == 2 ? 0 : q); };
  const cx<T>* in = static_cast<const cx<T>*>(a.in[0]);
  cx<T>* outb = static_cast<cx<T>*>(a.out[0]);
  const int lines = I.lines;
  cx<T> pre[2][4];
  // (where a wavefront's butterflies lie in one line, its line index is
  // wave-uniform and taken into scalar registers, so that the line
  // arithmetic and the row address run on the scalar unit)
  constexpr bool WU = sub >= 64;
  auto uni = [](int v) { return WU ? __builtin_amdgcn_readfirstlane(v) : v; };
  auto fetch = [&](int item) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int slot = uni(item * NL + bb + u * LPP);
      const bool ok = slot < lines;
      bool sh;
      const cx<T>* gin = in + (size_t)uni(ok ? mirror_line<true>(I, slot, &sh) : 0) * nt;
#pragma unroll
      for (int i = 0; i < 4; ++i) pre[u][i] = ok ? gin[ns(i)] : mk(T(0), T(0));
    }
  };
  constexpr int RL = PM::rad(PM::nst - 1), LRL = RL == 16 ? 4 : RL == 8 ? 3 : RL == 4 ? 2 : 1;
  constexpr int NB = 16 / RL;  // last-stage butterflies per thread
  constexpr int step = m / RL;
  constexpr int stepz = nz / PZ::rad(PZ::nst - 1);
  const double wsc = I.wcoef * I.scale;
  int item = blockIdx.x;
  if (item < a.total) fetch(item);
  for (; item < a.total; item += gridDim.x) {
    const int line0 = item * NL;
    const int nl = min(NL, lines - line0);
    // (the deconvolution factors and the first twiddle are read per item, not
    // held across it: the registers go to the later phases)
    T snr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) snr[i] = sn_at(ns(i));
    const cx<T> w1 = twm[j];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      cx<T> v[8];
      v[0] = cscl(pre[u][0], snr[0]);
      v[1] = cscl(pre[u][1], snr[1]);
      v[2] = v[3] = v[4] = v[5] = mk(T(0), T(0));
      v[6] = cscl(pre[u][2], snr[2]);
      v[7] = cscl(pre[u][3], snr[3]);
      dft_pow2<T, 8>(v);
      twiddle_pow2<T, 8>(v, w1);
      const int b = bb + u * LPP;
#pragma unroll
      for (int r = 0; r < 8; ++r) buf[pad(b * m + j + r * sub)] = v[r];
    }
    __syncthreads();
    p2_stages<T, LM, 1, p2_l16_m(LM), PADL, NT>(buf, twm, NL);
    if (item + (int)gridDim.x < a.total) fetch(item + gridDim.x);
    {
      // last grid stage, in place: read, barrier, write in natural order
      // (line b at buf + b LS, unpadded within its line)
      cx<T> lv[NB][RL];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int id = (int)threadIdx.x + u * NT;
        const int b = id >> (LM - LRL), blk = id & ((m >> LRL) - 1);
        const cx<T>* p = buf + pad(b * m + blk * RL);
#pragma unroll
        for (int r = 0; r < RL; ++r) lv[u][r] = p[r];
        dft_pow2<T, RL>(lv[u]);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int id = (int)threadIdx.x + u * NT;
        const int b = id >> (LM - LRL), blk = id & ((m >> LRL) - 1);
        cx<T>* g = buf + b * LS;
        const int k0 = PM::natural(blk * RL);
#pragma unroll
        for (int r = 0; r < RL; ++r) g[k0 + r * step] = lv[u][r];
      }
    }
    __syncthreads();
    {
      // interpolation (R: |l| = 1 .. nz/2, node pairs +-nu+): node pair p of
      // mirror pair h
      // (h is wave-uniform from half = 64 on)
      constexpr bool HU = half >= 64;
      auto hu = [](int v) { return HU ? __builtin_amdgcn_readfirstlane(v) : v; };
      const int h = hu((int)threadIdx.x >> (LZ - 1)), la = ((int)threadIdx.x & (half - 1)) + 1;
      const bool act = 2 * h < nl;
      cx<T> o[4] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
      if (act) {
        bool sh, sh1;
        const int L0 = hu(mirror_line<true>(I, line0 + 2 * h, &sh));
        const int L1 = hu(mirror_line<true>(I, line0 + 2 * h + 1, &sh1));
        const double bl = I.b * (double)la * (double)la;
        double nup = sqrt_nt(line_ak<true>(I, L0) + bl);
        // (the weight, halved on the Nyquist lane, rides on the node phase)
        const double wla = wsc * (double)la * (la < half ? 1.0 : 0.5);
        PairWin<T, TAPS> pw;
        pair_window<T, TAPS, true>(nup, I, a, m, 0.0, pw);
        pw.ph = cscl(pw.ph, T(wla * rcp_nt(nup)));
        cx<T> vp, vn;
        pair_values<T, TAPS, false>(buf + 2 * h * LS, m, pw, &vp, &vn);
        if (la < half) {
          o[0] = vp;
          o[1] = vn;
        } else {
          o[0] = cadd(vp, vn);
        }
        if (!sh) {
          nup = sqrt_nt(line_ak<true>(I, L1) + bl);
          pair_window<T, TAPS, true>(nup, I, a, m, 0.0, pw);
          pw.ph = cscl(pw.ph, T(wla * rcp_nt(nup)));
        }
        pair_values<T, TAPS, false>(buf + (2 * h + 1) * LS, m, pw, &vp, &vn);
        if (la < half) {
          o[2] = vp;
          o[3] = vn;
        } else {
          o[2] = cadd(vp, vn);
        }
      }
      __syncthreads();
      // the depth lines over the grid: line b at b nz (padded); the Nyquist
      // lane also writes l = 0 (weight 0)
      const int e0 = 2 * h * nz, e1 = e0 + nz;
      const int lp = la < half ? la : half, ln = la < half ? nz - la : 0;
      buf[pad(e0 + lp)] = cconj(o[0]);
      buf[pad(e0 + ln)] = cconj(o[1]);
      buf[pad(e1 + lp)] = cconj(o[2]);
      buf[pad(e1 + ln)] = cconj(o[3]);
    }
    __syncthreads();
    p2_stages<T, LZ, 0, p2_l16_z(LZ), PADL, NT>(buf, twz, NL);
    fft_last_stage_p2<T, PZ::rad(PZ::nst - 1), true, PADL, NT>(buf, nz, NL, nz, 1, [&](int b, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      if (b >= nl) return;
      bool sh;
      cx<T>* o = outb + (size_t)mirror_line<true>(I, line0 + b, &sh) * nz;
      const int k0 = PZ::natural(blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) o[k0 + r * stepz] = cconj(v[r]);
    });
    __syncthreads();
  }
}

// Fused depth DFT + spreading + transposed a2 (operators R^T and A).  A work
// item holds lpw_a lines: their depth DFTs run together (power-of-two
// builds: the first stage reads the spectra from memory and the last writes
// them in natural order), then each line is spread onto the grid and
// transformed back, and only its time line is stored.
template <typename T, int RS, int TAPS>
__global__ __launch_bounds__(kBlock) void k_line_nufft1(StageArgs a) {
  constexpr bool P2 = RS == 0;
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nz = I.nz, nt = I.nt;
  const int lpw = I.lpw_a;
  const int line0 = li * lpw;
  const int nl = min(lpw, I.lines - line0);
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;  // (global, as in k_line_nufft2)
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  const int sg = m > lpw * nz ? m : lpw * nz;
  cx<T>* grid = reinterpret_cast<cx<T>*>(pat_smem);  // depth-FFT scratch, then one grid line
  cx<T>* qn = grid + sg;                              // lpw depth spectra, natural order
  const SpreadLds<T, 2> L = SpreadLds<T, 2>::carve(qn + lpw * nz, nz, I.taps);
  const cx<T>* in = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)line0 * nz;
  if constexpr (P2) {
    const int stepz = nz / I.fz.rad[I.fz.nst - 1];  // weight of the last digit in k
    fft_lds_p2_src_sink<T, true>(
        grid, I.fz, twz, nl, nz, 1, [&](int b, int pos) { return in[(size_t)b * nz + pos]; },
        [&](int b, int blk, const auto& v) {
          constexpr int R = sizeof(v) / sizeof(v[0]);
          cx<T>* d = qn + b * nz;
          const int k0 = dif_natural_p2(I.fz, blk * R);
#pragma unroll
          for (int r = 0; r < R; ++r) d[k0 + r * stepz] = v[r];
        });
  } else {
    copy_batched<2>(nl * nz, [&](int e) { return in[e]; }, [&](int e, cx<T> v) { grid[e] = v; });
    __syncthreads();
    fft_lds<T, RS, true>(grid, I.fz, twz, nl, nz, 1);
    const int32_t* permz = I.perm + I.fz.perm;
    for (int e = threadIdx.x; e < nl * nz; e += kBlock) {
      int b, l;
      divmod<P2>(e, nz, &b, &l);
      qn[e] = grid[b * nz + permz[l]];
    }
    __syncthreads();
  }
  auto put = [&](int j, cx<T> v) { grid[j] = cconj(v); };
  auto put4 = [&](int j, const cx<T>* v) {
#pragma unroll
    for (int c = 0; c < 2; ++c) grid[j + c] = cconj(v[c]);
  };
  for (int b = 0; b < nl; ++b) {
    // (spread_line's first barrier also ends every read of the previous
    // line's grid)
    const cx<T>* qb = qn + b * nz;
    auto fget = [&](int l) { return qb[l]; };
    if (TAPS > 0 && a.pair_ok) {
      spread_line<T, (TAPS > 0 ? TAPS : 2), true>(I, a, line0 + b, a.mode, L, fget, put, put4);
    } else {
      spread_line<T, 0, false>(I, a, line0 + b, a.mode, L, fget, put, put4);
    }
    __syncthreads();
    ifft_pick_deconv<T, RS>(I, grid, 1, static_cast<cx<T>*>(a.out[inst_]) + (size_t)(line0 + b) * nt, twm);
  }
  PAT_END_ITEM
}

// k_line_nufft1 for m = 2^LM and nz = 2^LZ known at compile time (FP32,
// one instance): the same work, with both FFTs' stages fixed by P2Plan; the
// last stage of the grid FFT writes the picked, deconvolved samples straight
// to memory.  Five waves per SIMD (the register cap of 96 costs a 20-byte
// spill): the spreading is bound by instruction issue and gains more from
// the fifth wave than the spill takes.
template <typename T, int TAPS, int LM, int LZ>
__global__ __launch_bounds__(kBlock, 5) void k_line_nufft1_c(StageArgs a) {
  constexpr int m = 1 << LM, nz = 1 << LZ;
  using PM = P2Plan<LM>;  // (no radix-16 last stage: it spills at this kernel's register
  using PZ = P2Plan<LZ>;  // cap in the grid FFT and gained nothing in the depth FFT)
  static_assert(PM::nst >= 2 && PZ::nst >= 2, "two or more stages");
  PAT_FOR_EACH_ITEM(a)
  const int nt = I.nt;
  const int lpw = I.lpw_a;
  const int line0 = li * lpw;
  const int nl = min(lpw, I.lines - line0);
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  const int sg = m > lpw * nz ? m : lpw * nz;
  cx<T>* grid = reinterpret_cast<cx<T>*>(pat_smem);  // depth-FFT scratch, then one grid line
  cx<T>* qn = grid + sg;                              // lpw depth spectra, natural order
  const SpreadLds<T, 2> L = SpreadLds<T, 2>::carve(qn + lpw * nz, nz, I.taps);
  const cx<T>* in = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)line0 * nz;
  constexpr int stepz = nz / PZ::rad(PZ::nst - 1);
  fft_first_stage_p2<T, PZ::rad(0), true>(grid, nz, twz, nl, nz, 1,
                                          [&](int b, int pos) { return in[(size_t)b * nz + pos]; });
  __syncthreads();
  p2_stages<T, LZ, 1>(grid, twz, nl);
  fft_last_stage_p2<T, PZ::rad(PZ::nst - 1), true>(grid, nz, nl, nz, 1, [&](int b, int blk, const auto& v) {
    constexpr int R = sizeof(v) / sizeof(v[0]);
    cx<T>* d = qn + b * nz;
    const int k0 = PZ::natural(blk * R);
#pragma unroll
    for (int r = 0; r < R; ++r) d[k0 + r * stepz] = v[r];
  });
  __syncthreads();
  auto put = [&](int j, cx<T> v) { grid[j] = cconj(v); };
  auto put4 = [&](int j, const cx<T>* v) {
#pragma unroll
    for (int c = 0; c < 2; ++c) grid[j + c] = cconj(v[c]);
  };
  const T* sn = static_cast<const T*>(I.sn);
  constexpr int step = m / PM::rad(PM::nst - 1);
  for (int b = 0; b < nl; ++b) {
    const cx<T>* qb = qn + b * nz;
    auto fget = [&](int l) { return qb[l]; };
    if (TAPS > 0 && a.pair_ok) {
      spread_line<T, (TAPS > 0 ? TAPS : 2), true>(I, a, line0 + b, a.mode, L, fget, put, put4);
    } else {
      spread_line<T, 0, false>(I, a, line0 + b, a.mode, L, fget, put, put4);
    }
    __syncthreads();
    // X_n = s_n conj(G_k) for the natural index k = (n - nt/2) mod m
    cx<T>* x = static_cast<cx<T>*>(a.out[inst_]) + (size_t)(line0 + b) * nt;
    p2_stages<T, LM, 0>(grid, twm, 1);
    fft_last_stage_p2<T, PM::rad(PM::nst - 1), true>(grid, m, 1, m, 1, [&](int, int blk, const auto& v) {
      constexpr int R = sizeof(v) / sizeof(v[0]);
      const int k0 = PM::natural(blk * R);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n = (k0 + r * step + nt / 2) & (m - 1);
        if (n < nt) x[n] = cscl(cconj(v[r]), sn[n]);
      }
    });
  }
  PAT_END_ITEM
}

// The fused type-1 kernel with wavefront spreading (FP32 at four waves per
// SIMD, FP64 at two; m = 2^LM and nz = 2^LZ at compile time): a work item
// holds one line per wavefront.  The depth DFTs of its lines run together,
// then each wavefront spreads its line into its own grid line in LDS (no
// block barrier inside), and the grid DFTs of all lines run together; the
// last stage writes the picked, deconvolved samples to memory.  LDS: the
// lines' grids (also the depth-FFT scratch) and their depth spectra in
// natural order.
template <typename T, int TAPS, int LM, int LZ>
__global__ __launch_bounds__(kBlock, sizeof(T) == 4 ? 4 : 2) void k_line_nufft1_w(StageArgs a) {
  constexpr int m = 1 << LM, nz = 1 << LZ, NL = kBlock / 64;
  using PM = P2Plan<LM, p2_l16_m(LM)>;  // (radix-16 last stages, as in the type-2 kernel)
  using PZ = P2Plan<LZ, p2_l16_z(LZ)>;
  static_assert(PM::nst >= 2 && PZ::nst >= 2 && LZ <= LM, "two or more stages");
  cx<T>* grid = reinterpret_cast<cx<T>*>(pat_smem);  // NL grid lines (first the depth-FFT scratch)
  cx<T>* qn = grid + NL * m;                         // NL depth spectra, natural order
  PAT_FOR_EACH_ITEM(a)
  const int nt = I.nt;
  const int line0 = li * NL;
  const int nl = min(NL, I.lines - line0);
  const cx<T>* twm = static_cast<const cx<T>*>(I.tw) + I.fm.tw;
  const cx<T>* twz = static_cast<const cx<T>*>(I.tw) + I.fz.tw;
  const cx<T>* in = static_cast<const cx<T>*>(a.in[inst_]) + (size_t)line0 * nz;
  constexpr int stepz = nz / PZ::rad(PZ::nst - 1);
  fft_first_stage_p2<T, PZ::rad(0), true>(grid, nz, twz, nl, nz, 1,
                                          [&](int b, int pos) { return in[(size_t)b * nz + pos]; });
  __syncthreads();
  p2_stages<T, LZ, 1, p2_l16_z(LZ)>(grid, twz, nl);
  fft_last_stage_p2<T, PZ::rad(PZ::nst - 1), true>(grid, nz, nl, nz, 1, [&](int b, int blk, const auto& v) {
    constexpr int R = sizeof(v) / sizeof(v[0]);
    cx<T>* d = qn + b * nz;
    const int k0 = PZ::natural(blk * R);
#pragma unroll
    for (int r = 0; r < R; ++r) d[k0 + r * stepz] = v[r];
  });
  __syncthreads();
  const int wv = (int)(threadIdx.x >> 6);
  if (wv < nl) {
    const cx<T>* qb = qn + wv * nz;
    spread_line_wave<T, TAPS, true>(I, a, line0 + wv, a.mode, m, nz, grid + wv * m, [&](int l) { return qb[l]; });
  }
  __syncthreads();
  // X_n = s_n conj(G_k) for the natural index k = (n - nt/2) mod m
  const T* sn = static_cast<const T*>(I.sn);
  constexpr int step = m / PM::rad(PM::nst - 1);
  cx<T>* xout = static_cast<cx<T>*>(a.out[inst_]) + (size_t)line0 * nt;
  p2_stages<T, LM, 0, p2_l16_m(LM)>(grid, twm, nl);
  fft_last_stage_p2<T, PM::rad(PM::nst - 1), true>(grid, m, nl, m, 1, [&](int b, int blk, const auto& v) {
    constexpr int R = sizeof(v) / sizeof(v[0]);
    const int k0 = PM::natural(blk * R);
    cx<T>* x = xout + (size_t)b * nt;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = (k0 + r * step + nt / 2) & (m - 1);
      if (n < nt) x[n] = cscl(cconj(v[r]), sn[n]);
    }
  });
  PAT_END_ITEM
}

// Spreading alone with wavefront spreading (FP32 compute; grid stored as
// float or bf16 pairs): one line per wavefront, built in LDS and written out
// by the same wavefront with 16-byte stores.
template <typename G, int TAPS, bool P2>
__global__ __launch_bounds__(kBlock) void k_line_spread_w(StageArgs a) {
  constexpr int NL = kBlock / 64;
  PAT_FOR_EACH_ITEM(a)
  const int m = I.m, nz = I.nz;
  const int line0 = li * NL;
  const int wv = (int)(threadIdx.x >> 6), L = (int)(threadIdx.x & 63);
  if (line0 + wv < I.lines) {
    const int line = line0 + wv;
    cx<float>* Gl = reinterpret_cast<cx<float>*>(pat_smem) + wv * m;
    const cx<float>* F = static_cast<const cx<float>*>(a.in[inst_]) + (size_t)line * nz;
    spread_line_wave<float, TAPS, P2>(I, a, line, a.mode, m, nz, Gl, [&](int l) { return F[l]; });
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    G* row = static_cast<G*>(a.out[inst_]) + (size_t)line * m;
    for (int j = 4 * L; j < m; j += 4 * 64) {
      cx<float> v4[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) v4[c] = cconj(Gl[j + c]);
      grid_store4<float, G>(row + j, v4);
    }
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

// Workgroups of kBlock threads that one CU holds at once for this kernel and
// LDS size (cached: the query is not free and the answer never changes).
int resident_blocks(const void* kernel, size_t shmem, int block = kBlock) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kernel, shmem});
  if (it != cache.end()) return it->second;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, shmem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  cache[{kernel, shmem}] = per_cu;
  return per_cu;
}

// launches left before an injected failure (0: none); see set_launch_fault
thread_local int t_fault_countdown = 0;

// True when this launch is the one the PAT_FAULT hook fails.
bool launch_faulted() { return t_fault_countdown > 0 && --t_fault_countdown == 0; }

template <typename K>
hipError_t launch(K kernel, const char* name, StageArgs& a, size_t shmem, hipStream_t st, StageTimer* tm) {
  if (a.total <= 0) return hipSuccess;
  if (launch_faulted()) return hipErrorLaunchFailure;
  if (a.counter) {
    a.item_slot = (int32_t)((shmem + 15) & ~(size_t)15);
    shmem = (size_t)a.item_slot + 16;
  }
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  // one workgroup per item; with a work counter, a persistent grid of as many
  // workgroups as fit on the device at once
  const int cap = a.counter ? resident_blocks(reinterpret_cast<const void*>(kernel), shmem) * num_cu() : a.total;
  const int grid = a.total < cap ? a.total : cap;
  if (tm) tm->begin(name, st);
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), shmem, st, a);
  hipError_t e = hipGetLastError();
  if (tm) tm->end(st);
  return e;
}

// A persistent grid (as many workgroups as fit at once, at most one per item)
// for kernels that stride over their items themselves.
template <typename K>
hipError_t launch_persistent(K kernel, const char* name, StageArgs& a, size_t shmem, hipStream_t st,
                             StageTimer* tm, int block = kBlock) {
  if (a.total <= 0) return hipSuccess;
  if (launch_faulted()) return hipErrorLaunchFailure;
  if (shmem > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  const int cap = resident_blocks(reinterpret_cast<const void*>(kernel), shmem, block) * num_cu();
  const int grid = a.total < cap ? a.total : cap;
  if (tm) tm->begin(name, st);
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, st, a);
  hipError_t e = hipGetLastError();
  if (tm) tm->end(st);
  return e;
}

enum Items { IT_X1, IT_X2, IT_C2R, IT_LM, IT_LZ, IT_LI, IT_LF, IT_LA, IT_LINE, IT_LWAVE };

int cdiv(int a, int b) { return (a + b - 1) / b; }

int items_of(const Inst& I, Items kind, bool nz) {
  const int len = nz ? I.nz : I.nt;
  switch (kind) {
    case IT_X1: return I.n2 * cdiv(len, 2 * I.tb);
    case IT_X2: return I.n2 > 1 ? I.h1 * cdiv(len, I.tb) : 0;
    case IT_C2R: return I.n2 * cdiv(len, 2 * I.tb);
    case IT_LM: return cdiv(I.lines, I.lpw_m);
    case IT_LZ: return cdiv(I.lines, I.lpw_z);
    case IT_LI: return cdiv(I.lines, I.lpw_i);
    case IT_LF: return cdiv(I.lines, I.lpw_f);
    case IT_LA: return cdiv(I.lines, I.lpw_a);
    case IT_LINE: return I.lines;
    case IT_LWAVE: return cdiv(I.lines, kBlock / 64);  // one line per wavefront
  }
  return 0;
}

template <typename T, typename G, int RS, int TAPS>
struct Runner {
  static constexpr bool P2 = RS == 0;
  int n;
  const Inst* h;
  const Inst* const* d;
  const void* const* hp;  // host tap-polynomial tables
  uint32_t* counters;
  int next_counter;
  hipStream_t st;
  StageTimer* tm;

  static constexpr size_t cs = sizeof(cx<T>);

  StageArgs base(Items kind, bool nz, int mode, const void* const* in, void* const* out) {
    StageArgs a;
    a.n = n;
    a.len_nz = nz ? 1 : 0;
    a.mode = mode;
    a.off[0] = 0;
    for (int i = 0; i < n; ++i) {
      a.inst[i] = d[i];
      a.in[i] = in[i];
      a.out[i] = out[i];
      a.off[i + 1] = a.off[i] + items_of(h[i], kind, nz);
    }
    a.total = a.off[n];
    a.counter = counters ? counters + (next_counter++ % kNumCounters) : nullptr;
    fill_pairs(a);
    return a;
  }

  // Mirrored tap-pair coefficients into the arguments when every instance
  // uses the same fitted table with TAPS (even) taps.
  void fill_pairs(StageArgs& a) const {
    a.pair_ok = 0;
    constexpr int D = Deg<T>::v, D1 = D + 1, NE = D / 2 + 1, NO = (D + 1) / 2, PW = NE + NO;
    if (TAPS <= 0 || TAPS % 2 != 0 || (size_t)(TAPS / 2) * PW * sizeof(T) > sizeof(a.pc) || !hp) return;
    for (int i = 0; i < n; ++i) {
      if (!h[i].poly || h[i].taps != TAPS || !hp[i]) return;
      if (std::memcmp(hp[i], hp[0], (size_t)TAPS * D1 * sizeof(T)) != 0) return;
    }
    const T* mono = static_cast<const T*>(hp[0]);
    T pc[(TAPS > 0 ? TAPS / 2 : 1) * PW];
    for (int p = 0; p < TAPS / 2; ++p) {
      for (int e = 0; e < NE; ++e) pc[p * PW + e] = mono[p * D1 + 2 * e];
      for (int o = 0; o < NO; ++o) pc[p * PW + NE + o] = mono[p * D1 + 2 * o + 1];
    }
    std::memcpy(a.pc, pc, sizeof(pc));
    a.pair_ok = 1;
  }

  template <typename F>
  size_t max_over(F f) const {
    size_t mx = 0;
    for (int i = 0; i < n; ++i) {
      const size_t v = f(h[i]);
      if (v > mx) mx = v;
    }
    return mx;
  }

  // The pipelined transverse kernels run for one instance; lengths of 128,
  // 256 and 512 points with the plan's tile width take the compile-time
  // instances (FP64 only these: its run-time-size pipelines, sized for the
  // largest tile, would spill), other FP32 lengths the run-time-size ones.
  hipError_t x1(const void* const* in, void* const* out, bool nz) {
    StageArgs a = base(IT_X1, nz, 0, in, out);
    const int len = nz ? h[0].nz : h[0].nt;
    {
      if (n == 1 && !a.counter && len % 4 == 0 && h[0].tb % 2 == 0 && h[0].n1 * (h[0].tb / 2) <= kPipeU * kBlock) {
        const size_t ew = (size_t)(h[0].cut_e + 1) * (h[0].cut_e + 1);
        const size_t shm = (size_t)h[0].n1 * (h[0].tb + 1) * cs + (size_t)((h[0].n1 + 3) & ~3) * sizeof(int32_t) +
                           (!nz && h[0].cut_e ? 2 * ew * sizeof(T) : 0);
        auto go = [&](auto kern) { return launch_persistent(kern, "dft_x1", a, shm, st, tm); };
        if constexpr (RS == 0) {
          const int L = h[0].n1, tb = h[0].tb;
          if (L == 128 && tb == pipe_tb<T>(7)) return go(k_tr_x1_pipe<T, RS, 7>);
          if (L == 256 && tb == pipe_tb<T>(8)) return go(k_tr_x1_pipe<T, RS, 8>);
          if (L == 512 && tb == pipe_tb<T>(9)) return go(k_tr_x1_pipe<T, RS, 9>);
        }
        if constexpr (sizeof(T) == 4) return go(k_tr_x1_pipe<T, RS>);
      }
    }
    return launch(k_tr_x1_r2c<T, RS>, "dft_x1", a, max_over([](const Inst& I) { return lds_tile_x1(I, cs); }), st,
                  tm);
  }
  hipError_t x2(void* const* io, bool nz, int inv) {
    StageArgs a = base(IT_X2, nz, inv, io, io);
    const char* name = inv ? "idft_x2" : "dft_x2";
    {
      if (n == 1 && !a.counter && h[0].tb % 2 == 0 && h[0].n2 * (h[0].tb / 2) <= kPipeU * kBlock) {
        const size_t shm = lds_tile_x2(h[0], cs) + (size_t)((h[0].n2 + 3) & ~3) * sizeof(int32_t);
        auto go = [&](auto kern) { return launch_persistent(kern, name, a, shm, st, tm); };
        if constexpr (RS == 0) {
          const int L = h[0].n2, tb = h[0].tb;
          if (L == 128 && tb == pipe_tb<T>(7)) return go(k_tr_x2_pipe<T, RS, 7>);
          if (L == 256 && tb == pipe_tb<T>(8)) return go(k_tr_x2_pipe<T, RS, 8>);
          if (L == 512 && tb == pipe_tb<T>(9)) return go(k_tr_x2_pipe<T, RS, 9>);
        }
        if constexpr (sizeof(T) == 4) return go(k_tr_x2_pipe<T, RS>);
      }
    }
    return launch(k_tr_x2<T, RS>, name, a, max_over([](const Inst& I) { return lds_tile_x2(I, cs); }), st, tm);
  }
  hipError_t c2r(const void* const* in, void* const* out, bool nz) {
    StageArgs a = base(IT_C2R, nz, 0, in, out);
    const int len = nz ? h[0].nz : h[0].nt;
    {
      if (n == 1 && !a.counter && !(!nz && h[0].cut_e) && len % 4 == 0 && h[0].tb % 2 == 0 &&
          h[0].n1 * h[0].tb <= 2 * kPipeU * kBlock) {
        const size_t shm = (size_t)h[0].n1 * (h[0].tb + 1) * cs + (size_t)((h[0].n1 + 3) & ~3) * sizeof(int32_t);
        auto go = [&](auto kern) { return launch_persistent(kern, "idft_x1_c2r", a, shm, st, tm); };
        if constexpr (RS == 0) {
          const int L = h[0].n1, tb = h[0].tb;
          if (L == 128 && tb == pipe_tb<T>(7)) return go(k_tr_c2r_pipe<T, RS, 7>);
          if (L == 256 && tb == pipe_tb<T>(8)) return go(k_tr_c2r_pipe<T, RS, 8>);
          if (L == 512 && tb == pipe_tb<T>(9)) return go(k_tr_c2r_pipe<T, RS, 9>);
        }
        if constexpr (sizeof(T) == 4) return go(k_tr_c2r_pipe<T, RS>);
      }
    }
    return launch(k_tr_c2r_k1<T, RS>, "idft_x1_c2r", a, max_over([](const Inst& I) { return lds_tile_x1(I, cs); }),
                  st, tm);
  }
  hipError_t zfft(void* const* io, int inv) {
    StageArgs a = base(IT_LZ, true, inv, io, io);
    return launch(k_line_fft<T, RS>, inv ? "idft_z" : "dft_z", a,
                  max_over([](const Inst& I) { return lds_line_z(I, cs); }), st, tm);
  }
  hipError_t a2(const void* const* in, void* const* out) {
    StageArgs a = base(IT_LM, false, 0, in, out);
    if constexpr (sizeof(T) == 4 && P2) {
      // one instance, centred c = 2 grid, m = 2^8 .. 2^11: the pipelined kernel
      const Inst& I = h[0];
      const int lm = __builtin_ctz((unsigned)I.m);
      if (n == 1 && !a.counter && I.centred && I.m == 2 * I.nt && lm >= 8 && lm <= 11 && I.fm.rad[0] == 8 &&
          I.lpw_m == 2048 / I.m) {
        const size_t shm = (size_t)(2048 + 2048 + 2048 / 16) * cs;
        auto go = [&](auto kern) { return launch_persistent(kern, "deconv_pad_fft", a, shm, st, tm); };
        if (lm == 8) return go(k_line_a2_pipe<G, 8>);
        if (lm == 9) return go(k_line_a2_pipe<G, 9>);
        if (lm == 10) return go(k_line_a2_pipe<G, 10>);
        return go(k_line_a2_pipe<G, 11>);
      }
    }
    return launch(k_line_a2<T, G, RS>, "deconv_pad_fft", a, max_over([](const Inst& I) { return lds_line_m(I, cs); }),
                  st, tm);
  }
  hipError_t a2t(const void* const* in, void* const* out) {
    StageArgs a = base(IT_LM, false, 0, in, out);
    if constexpr (sizeof(T) == 4 && P2) {
      // one instance, centred c = 2 grid, m = 2^8 .. 2^11: the pipelined kernel
      const Inst& I = h[0];
      const int lm = __builtin_ctz((unsigned)I.m);
      if (n == 1 && !a.counter && I.centred && I.m == 2 * I.nt && lm >= 8 && lm <= 11 && I.lpw_m == 2048 / I.m) {
        const size_t shm = (size_t)(2048 + 2048 / 16) * cs;
        auto go = [&](auto kern) { return launch_persistent(kern, "ifft_pick_deconv", a, shm, st, tm); };
        if (lm == 8) return go(k_line_a2t_pipe<G, 8>);
        if (lm == 9) return go(k_line_a2t_pipe<G, 9>);
        if (lm == 10) return go(k_line_a2t_pipe<G, 10>);
        return go(k_line_a2t_pipe<G, 11>);
      }
    }
    return launch(k_line_a2t<T, G, RS>, "ifft_pick_deconv", a,
                  max_over([](const Inst& I) { return lds_line_m(I, cs); }), st, tm);
  }
  hipError_t interp(const void* const* in, void* const* out, int mode) {
    StageArgs a = base(IT_LI, true, mode, in, out);
    if constexpr (TAPS > 0) {
      // one instance with the paired taps: the streamed kernel, with enough
      // 16-byte registers per thread for a line group
      constexpr int EPC = GridChunk<T, G>::EPC;
      const Inst& I = h[0];
      const int per = (I.lpw_i * I.m / EPC + kBlock - 1) / kBlock;
      if (n == 1 && a.pair_ok && I.m % EPC == 0 && per <= 8 && !counters) {
        const size_t shm = lds_interp_stream(I, cs);
        if (per <= 1) return launch_persistent(k_line_interp_stream<T, G, TAPS, P2, 1>, "interp", a, shm, st, tm);
        if (per <= 2) return launch_persistent(k_line_interp_stream<T, G, TAPS, P2, 2>, "interp", a, shm, st, tm);
        if (per <= 4) return launch_persistent(k_line_interp_stream<T, G, TAPS, P2, 4>, "interp", a, shm, st, tm);
        return launch_persistent(k_line_interp_stream<T, G, TAPS, P2, 8>, "interp", a, shm, st, tm);
      }
    }
    return launch(k_line_interp<T, G, TAPS, P2>, "interp", a,
                  max_over([](const Inst& I) { return lds_interp(I, cs); }), st, tm);
  }
  hipError_t spread(const void* const* in, void* const* out, int mode) {
    if constexpr (sizeof(T) == 4 && TAPS > 0 && TAPS % 2 == 0) {
      // FP32 with the paired taps: one line per wavefront (its grid line in
      // LDS, up to 2048 points)
      StageArgs a = base(IT_LWAVE, true, mode, in, out);
      const size_t shm = max_over([](const Inst& I) { return lds_spread_wave(I); });
      bool ok = a.pair_ok && shm <= 65536;
      for (int i = 0; i < n; ++i) ok = ok && h[i].m % 4 == 0;
      if (ok) return launch(k_line_spread_w<G, TAPS, P2>, "spread", a, shm, st, tm);
      next_counter--;  // (the counter taken by base() above is not used)
    }
    StageArgs a = base(IT_LINE, true, mode, in, out);
    return launch(k_line_spread<T, G, TAPS>, "spread", a,
                  max_over([](const Inst& I) { return lds_spread(I, cs); }), st, tm);
  }
  hipError_t nufft2(const void* const* in, void* const* out, int mode) {
    StageArgs a = base(IT_LF, true, mode, in, out);
    if constexpr (P2 && TAPS > 0) {
      const Inst& I = h[0];
      if (n == 1 && !a.counter && a.pair_ok && mode == 0 && I.m == 2 * I.nt && 4 * I.nz == I.m && I.n2 >= 4 &&
          I.fm.nst >= 2 && I.fm.rad[0] == 8) {
        // R on 3D plans with nz = m/4: line groups in mirror pairs, m = 2^8 .. 2^11
        const int lm = __builtin_ctz((unsigned)I.m);
        if (lm >= 8 && lm <= 11) {
          // two waves per workgroup up to m = 1024 (one mirror pair there),
          // four at m = 2048
          const int nt_ = lm <= 10 ? 128 : 256;
          a.total = cdiv(I.lines, 16 * nt_ / I.m);
          a.off[1] = a.total;
          auto go = [&](auto kern, int shm) { return launch_persistent(kern, "nufft_fused", a, shm, st, tm, nt_); };
          if (lm == 8) return go(k_line_nufft2_mirror<T, TAPS, 8, 6, 128>, MirrorLds<T, 8, 128>::bytes);
          if (lm == 9) return go(k_line_nufft2_mirror<T, TAPS, 9, 7, 128>, MirrorLds<T, 9, 128>::bytes);
          if (lm == 10) return go(k_line_nufft2_mirror<T, TAPS, 10, 8, 128>, MirrorLds<T, 10, 128>::bytes);
          return go(k_line_nufft2_mirror<T, TAPS, 11, 9, 256>, MirrorLds<T, 11, 256>::bytes);
        }
      }
    }
    if constexpr (P2 && TAPS > 0) {
      // FP32, and FP64 at two waves per SIMD (its launch bound)
      const Inst& I = h[0];
      if (n == 1 && !a.counter && a.pair_ok && I.m == 2 * I.nt && I.m >= I.nz && I.fm.nst >= 2 &&
          I.fm.rad[0] == 8 && (I.m / 8) * I.lpw_f == kBlock) {
        // compile-time sizes for m = 2^8 .. 2^11 and nz = m/4 or m/2 (with
        // the padded scratch)
        const size_t shm = lds_fused2(I, cs) + (size_t)I.lpw_f * (I.m / 16) * cs;
        const int lm = __builtin_ctz((unsigned)I.m), dz = lm - __builtin_ctz((unsigned)I.nz);
        auto go = [&](auto kern) { return launch_persistent(kern, "nufft_fused", a, shm, st, tm); };
        if (dz == 2) {
          if (lm == 8) return go(k_line_nufft2_pipe_c<T, TAPS, 8, 6>);
          if (lm == 9) return go(k_line_nufft2_pipe_c<T, TAPS, 9, 7>);
          if (lm == 10) return go(k_line_nufft2_pipe_c<T, TAPS, 10, 8>);
          if (lm == 11) return go(k_line_nufft2_pipe_c<T, TAPS, 11, 9>);
        } else if (dz == 1) {
          if (lm == 8) return go(k_line_nufft2_pipe_c<T, TAPS, 8, 7>);
          if (lm == 9) return go(k_line_nufft2_pipe_c<T, TAPS, 9, 8>);
          if (lm == 10) return go(k_line_nufft2_pipe_c<T, TAPS, 10, 9>);
          if (lm == 11) return go(k_line_nufft2_pipe_c<T, TAPS, 11, 10>);
        }
        if constexpr (sizeof(T) == 4) return go(k_line_nufft2_pipe<T, TAPS>);
      }
    }
    return launch(k_line_nufft2<T, RS, TAPS>, "nufft_fused", a,
                  max_over([](const Inst& I) { return lds_fused2(I, cs); }), st, tm);
  }
  hipError_t nufft1(const void* const* in, void* const* out, int mode) {
    if constexpr (P2 && TAPS > 0 && TAPS % 2 == 0) {
      // one line per wavefront, compile-time sizes for m = 2^8 .. 2^10 and
      // nz = m/4 or m/2
      const Inst& I = h[0];
      const int lm = __builtin_ctz((unsigned)I.m), dz = lm - __builtin_ctz((unsigned)I.nz);
      StageArgs a = base(IT_LWAVE, true, mode, in, out);
      if (n == 1 && a.pair_ok && (dz == 1 || dz == 2) && lm >= 8 && lm <= 10) {
        const size_t shm = lds_fused1_wave(I, cs);
        auto go = [&](auto kern) { return launch(kern, "nufft_adjoint_fused", a, shm, st, tm); };
        if (dz == 2) {
          if (lm == 8) return go(k_line_nufft1_w<T, TAPS, 8, 6>);
          if (lm == 9) return go(k_line_nufft1_w<T, TAPS, 9, 7>);
          return go(k_line_nufft1_w<T, TAPS, 10, 8>);
        }
        if (lm == 8) return go(k_line_nufft1_w<T, TAPS, 8, 7>);
        if (lm == 9) return go(k_line_nufft1_w<T, TAPS, 9, 8>);
        return go(k_line_nufft1_w<T, TAPS, 10, 9>);
      }
      next_counter--;
    }
    StageArgs a = base(IT_LA, true, mode, in, out);
    if constexpr (sizeof(T) == 4 && P2 && TAPS > 0) {
      // compile-time sizes for m = 2^8 .. 2^11 and nz = m/4 or m/2
      const Inst& I = h[0];
      const int lm = __builtin_ctz((unsigned)I.m), dz = lm - __builtin_ctz((unsigned)I.nz);
      const size_t shm = lds_fused1(I, cs);
      auto go = [&](auto kern) { return launch(kern, "nufft_adjoint_fused", a, shm, st, tm); };
      if (n == 1 && dz == 2) {
        if (lm == 8) return go(k_line_nufft1_c<T, TAPS, 8, 6>);
        if (lm == 9) return go(k_line_nufft1_c<T, TAPS, 9, 7>);
        if (lm == 10) return go(k_line_nufft1_c<T, TAPS, 10, 8>);
        if (lm == 11) return go(k_line_nufft1_c<T, TAPS, 11, 9>);
      } else if (n == 1 && dz == 1) {
        if (lm == 8) return go(k_line_nufft1_c<T, TAPS, 8, 7>);
        if (lm == 9) return go(k_line_nufft1_c<T, TAPS, 9, 8>);
        if (lm == 10) return go(k_line_nufft1_c<T, TAPS, 10, 9>);
        if (lm == 11) return go(k_line_nufft1_c<T, TAPS, 11, 10>);
      }
    }
    return launch(k_line_nufft1<T, RS, TAPS>, "nufft_adjoint_fused", a,
                  max_over([](const Inst& I) { return lds_fused1(I, cs); }), st, tm);
  }
};

#define PAT_TRY(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

template <typename T, typename G, int RS, int TAPS>
hipError_t run_op_t(Op op, int stage, int n, const Inst* h, const Inst* const* d, const void* const* hp,
                    const void* const* in, void* const* out, void* const* ws, uint32_t* counters, int counter0,
                    hipStream_t st, StageTimer* tm) {
  // stage s (1 .. 5) of the operator; the persistent launches of a stage
  // take work counters from counter0 on (stage 3 may launch three kernels)
  static const int kCounterAt[6] = {0, 0, 1, 2, 5, 6};
  Runner<T, G, RS, TAPS> r{n, h, d, hp, counters, counter0 + kCounterAt[stage], st, tm};
  void* bg[kMaxBatch];
  void* bu[kMaxBatch];
  void* bf[kMaxBatch];
  bool fused = true;
  for (int i = 0; i < n; ++i) {
    char* w = static_cast<char*>(ws[i]);
    bg[i] = w + h[i].off_g;
    bu[i] = w + h[i].off_u;
    bf[i] = w + h[i].off_f;
    fused = fused && h[i].fused;
  }
  const bool fwd = op == OP_R || op == OP_AT;  // type-2 line stage (else type-1)
  void* const* a = fwd ? bg : bf;               // the transverse spectrum of the input
  void* const* b = fwd ? bf : bg;               // the transverse spectrum of the output
  const int mode = (op == OP_R || op == OP_RT) ? 0 : 1;
  switch (stage) {
    case 1: return r.x1(in, a, !fwd);
    case 2: return r.x2(a, !fwd, 0);
    case 3:
      if (fwd) {
        if (fused) return r.nufft2(bg, bf, mode);
        PAT_TRY(r.a2(bg, bu));
        PAT_TRY(r.interp(bu, bf, mode));
        return r.zfft(bf, 1);
      }
      if (fused) return r.nufft1(bf, bg, mode);
      PAT_TRY(r.zfft(bf, 0));
      PAT_TRY(r.spread(bf, bu, mode));
      return r.a2t(bu, bg);
    case 4: return r.x2(b, fwd, 1);
    case 5: return r.c2r(b, out, fwd);
  }
  return hipSuccess;
}

bool all_pow2(int n, const Inst* h) {
  for (int i = 0; i < n; ++i)
    if (!h[i].pow2) return false;
  return true;
}

// Largest radix over every FFT of the instances.
int max_radix(int n, const Inst* h) {
  int mx = 2;
  for (int i = 0; i < n; ++i) {
    for (const FftDesc* f : {&h[i].f1, &h[i].f2, &h[i].fm, &h[i].fz})
      for (int s = 0; s < f->nst; ++s) mx = f->rad[s] > mx ? f->rad[s] : mx;
  }
  return mx;
}

bool all_taps(int n, const Inst* h, int taps) {
  for (int i = 0; i < n; ++i)
    if (h[i].taps != taps) return false;
  return true;
}

// Stage `stage` of an operator over n instances with one kernel build (the
// radix set of their largest prime).
template <typename T, typename G>
hipError_t dispatch_one_build(Op op, int stage, int n, const Inst* h, const Inst* const* d, const void* const* hp,
                              const void* const* in, void* const* out, void* const* ws, uint32_t* counters,
                              int counter0, hipStream_t st, StageTimer* tm) {
  const bool t12 = all_taps(n, h, 12);
  if (all_pow2(n, h)) {
    if (t12) return run_op_t<T, G, 0, 12>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
    return run_op_t<T, G, 0, 0>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
  }
  if (max_radix(n, h) <= 8) {
    if (t12) return run_op_t<T, G, 7, 12>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
    return run_op_t<T, G, 7, 0>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
  }
  if (t12) return run_op_t<T, G, 23, 12>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
  return run_op_t<T, G, 23, 0>(op, stage, n, h, d, hp, in, out, ws, counters, counter0, st, tm);
}

// The radix class of an instance's FFT lengths: 0 powers of two, 1 radices up
// to 8, 2 larger primes (the kernel build each class needs).
int radix_class(const Inst& I) {
  if (I.pow2) return 0;
  return max_radix(1, &I) <= 8 ? 1 : 2;
}

// An operator over n instances.  Several instances are grouped by radix
// class, so that every instance runs the kernel build its own lengths need
// (one build over all would give every instance the registers of the largest
// prime's butterflies); each stage then runs one persistent launch per class
// present, all classes' stage s before any class's stage s + 1, so that only
// the last stage writes the outputs.  A class of one instance takes the
// single-instance kernels.  The work counters are cleared once, up front.
template <typename T, typename G>
hipError_t dispatch(Op op, int n, const Inst* h, const Inst* const* d, const void* const* hp, const void* const* in,
                    void* const* out, void* const* ws, uint32_t* counters, hipStream_t st, StageTimer* tm,
                    const ForkStreams* fork) {
  if (counters) {
    if (launch_faulted()) return hipErrorLaunchFailure;
    if (tm) tm->begin("zero_counters", st);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counters, kNumCounters);
    PAT_TRY(hipGetLastError());
    if (tm) tm->end(st);
  }
  if (n == 1) {
    for (int stage = 1; stage <= 5; ++stage) {
      const hipError_t e = dispatch_one_build<T, G>(op, stage, 1, h, d, hp, in, out, ws, counters, 0, st, tm);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  struct Group {
    int k = 0;
    Inst h[kMaxBatch];
    const Inst* d[kMaxBatch];
    const void* hp[kMaxBatch];
    const void* in[kMaxBatch];
    void* out[kMaxBatch];
    void* ws[kMaxBatch];
  };
  static thread_local Group g[3];
  for (int c = 0; c < 3; ++c) g[c].k = 0;
  for (int i = 0; i < n; ++i) {
    Group& G_ = g[radix_class(h[i])];
    const int k = G_.k++;
    G_.h[k] = h[i];
    G_.d[k] = d[i];
    G_.hp[k] = hp[i];
    G_.in[k] = in[i];
    G_.out[k] = out[i];
    G_.ws[k] = ws[i];
  }
  // With the plan's fork streams (and no timer), each class after the first
  // runs on a stream of its own, forked from st after the counters are
  // cleared and joined back into st at the end, so that one class's launch
  // tails overlap another's work.  The host enqueues in the same order.
  int ncls = 0;
  for (int c = 0; c < 3; ++c) ncls += g[c].k > 0 ? 1 : 0;
  const bool forked = fork && !tm && ncls > 1;
  hipStream_t cs[3] = {st, st, st};
  if (forked) {
    PAT_TRY(hipEventRecord(fork->ev[0], st));
    int j = 0;
    bool first = true;
    for (int c = 0; c < 3; ++c) {
      if (g[c].k == 0) continue;
      if (first) {
        first = false;
        continue;
      }
      cs[c] = fork->s[j++];
      PAT_TRY(hipStreamWaitEvent(cs[c], fork->ev[0], 0));
    }
  }
  hipError_t e = hipSuccess;
  for (int stage = 1; stage <= 5 && e == hipSuccess; ++stage) {
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
      if (g[c].k == 0) continue;
      e = dispatch_one_build<T, G>(op, stage, g[c].k, g[c].h, g[c].d, g[c].hp, g[c].in, g[c].out, g[c].ws,
                                   g[c].k == 1 ? nullptr : counters, 8 * c, cs[c], tm);
    }
  }
  if (forked) {
    // (joined also after a failed launch: st then orders after everything
    // that was enqueued)
    int j = 1;
    for (int c = 0; c < 3; ++c) {
      if (cs[c] == st) continue;
      const hipError_t r = hipEventRecord(fork->ev[j], cs[c]);
      const hipError_t w = r == hipSuccess ? hipStreamWaitEvent(st, fork->ev[j], 0) : r;
      if (e == hipSuccess) e = w;
      ++j;
    }
  }
  return e;
}

template <typename T, typename G>
hipError_t interp_only(const Inst& h, const Inst* dinst, const void* hpoly, const void* grid, void* out,
                       hipStream_t st, StageTimer* tm) {
  const Inst* d[1] = {dinst};
  const void* hp[1] = {hpoly};
  const void* in[1] = {grid};
  void* o[1] = {out};
  if (h.taps == 12) {
    if (h.pow2) {
      Runner<T, G, 0, 12> r{1, &h, d, hp, nullptr, 0, st, tm};
      return r.interp(in, o, 0);
    }
    Runner<T, G, 23, 12> r{1, &h, d, hp, nullptr, 0, st, tm};
    return r.interp(in, o, 0);
  }
  Runner<T, G, 23, 0> r{1, &h, d, hp, nullptr, 0, st, tm};
  return r.interp(in, o, 0);
}

template <typename T, typename G>
hipError_t spread_only(const Inst& h, const Inst* dinst, const void* hpoly, const void* vals, void* grid,
                       hipStream_t st, StageTimer* tm) {
  const Inst* d[1] = {dinst};
  const void* hp[1] = {hpoly};
  const void* in[1] = {vals};
  void* o[1] = {grid};
  if (h.taps == 12) {
    if (h.pow2) {
      Runner<T, G, 0, 12> r{1, &h, d, hp, nullptr, 0, st, tm};
      return r.spread(in, o, 0);
    }
    Runner<T, G, 23, 12> r{1, &h, d, hp, nullptr, 0, st, tm};
    return r.spread(in, o, 0);
  }
  Runner<T, G, 23, 0> r{1, &h, d, hp, nullptr, 0, st, tm};
  return r.spread(in, o, 0);
}

}  // namespace

hipError_t run_op(int prec, Op op, int n, const Inst* hinst, const Inst* const* dinst, const void* const* hpoly,
                  const void* const* in, void* const* out, void* const* ws, uint32_t* counters, hipStream_t stream,
                  StageTimer* timer, const ForkStreams* fork) {
  switch (prec) {
    case PREC_F64:
      return dispatch<double, cx<double>>(op, n, hinst, dinst, hpoly, in, out, ws, counters, stream, timer, fork);
    case PREC_F32:
      return dispatch<float, cx<float>>(op, n, hinst, dinst, hpoly, in, out, ws, counters, stream, timer, fork);
    case PREC_BF16:
      return dispatch<float, bf2>(op, n, hinst, dinst, hpoly, in, out, ws, counters, stream, timer, fork);
  }
  return hipErrorInvalidValue;
}

hipError_t run_interp(int prec, const Inst& hinst, const Inst* dinst, const void* hpoly, const void* grid, void* out,
                      hipStream_t stream, StageTimer* timer) {
  switch (prec) {
    case PREC_F64: return interp_only<double, cx<double>>(hinst, dinst, hpoly, grid, out, stream, timer);
    case PREC_F32: return interp_only<float, cx<float>>(hinst, dinst, hpoly, grid, out, stream, timer);
    case PREC_BF16: return interp_only<float, bf2>(hinst, dinst, hpoly, grid, out, stream, timer);
  }
  return hipErrorInvalidValue;
}

// Workspace of the allocation-free entry point: one array per device, held
// until the process ends.  Host code never passes `scratch` itself (on the
// host it is only a stand-in for the symbol): kernels get the device address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void set_launch_fault(int k) { t_fault_countdown = k > 0 ? k : 0; }

hipError_t scratch_buffer(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t run_spread(int prec, const Inst& hinst, const Inst* dinst, const void* hpoly, const void* vals, void* grid,
                      hipStream_t stream, StageTimer* timer) {
  switch (prec) {
    case PREC_F64: return spread_only<double, cx<double>>(hinst, dinst, hpoly, vals, grid, stream, timer);
    case PREC_F32: return spread_only<float, cx<float>>(hinst, dinst, hpoly, vals, grid, stream, timer);
    case PREC_BF16: return spread_only<float, bf2>(hinst, dinst, hpoly, vals, grid, stream, timer);
  }
  return hipErrorInvalidValue;
}

}  // namespace pat
