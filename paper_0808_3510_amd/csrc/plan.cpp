// Host-side plan: geometry validation and the FP64 constant tables
// (deconvolution factors, FFT twiddles and index maps, node/weight constants).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

namespace pat {

namespace {


size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Radices for an in-place DIF transform of length L: eights for the powers of
// two (a 2 or 4 absorbed as 4 or 4*4), then the odd primes.  Empty for L = 1.
bool factorize(int L, std::vector<int>* rad) {
  rad->clear();
  int e = 0;
  while (L % 2 == 0) {
    L /= 2;
    ++e;
  }
  int n8 = e / 3;
  const int rem = e % 3;
  std::vector<int> small;
  if (rem == 1) {
    if (n8 > 0) {
      --n8;
      small = {4, 4};
    } else {
      small = {2};
    }
  } else if (rem == 2) {
    small = {4};
  }
  for (int i = 0; i < n8; ++i) rad->push_back(8);
  for (int r : small) rad->push_back(r);
  static const int odd[] = {3, 5, 7, 11, 13, 17, 19, 23};
  for (int p : odd) {
    while (L % p == 0) {
      L /= p;
      rad->push_back(p);
    }
  }
  return L == 1 && (int)rad->size() <= kMaxStages;
}

// Position of natural-order bin k after the in-place DIF transform:
// k = d1 + R1 (d2 + R2 (...)),  pos = sum_i d_i L / (R1 ... Ri).
std::vector<int32_t> dif_positions(int L, const std::vector<int>& rad) {
  std::vector<int32_t> pos(L);
  for (int k = 0; k < L; ++k) {
    int rest = k, span = L, p = 0;
    for (int r : rad) {
      span /= r;
      p += (rest % r) * span;
      rest /= r;
    }
    pos[k] = p;
  }
  return pos;
}

// The interpolation kernel of the tap loop (see kernels.hip, kb_phi):
// Psi_hat(u) I0(alpha K) / (2 e^{alpha K}) = e^{alpha (s - K)} (1 - e^{-2 alpha s}) / (2 s).
double kb_phi_host(double u, double K, double a) {
  double s2 = (K - u) * (K + u);
  if (s2 < 0) s2 = 0;
  const double s = std::sqrt(s2);
  const double as = a * s;
  const double v = as > 1e-3 ? -std::expm1(-2.0 * as) / (2.0 * s) : a * (1.0 - as + 2.0 / 3.0 * as * as);
  return std::exp(a * (s - K)) * v;
}

// Tap t of a node with fractional offset delta in (cK - 1, cK] weighs
// phi((delta - t)/c).  Writing delta = cK - 1/2 + x/2, x in (-1, 1], each tap
// is a smooth function of x; it is interpolated at the D+1 Chebyshev points
// and stored in monomial form.  Returns the largest error on a fine grid
// relative to the largest tap value.
double fit_tap_polys(double c, double K, double a, int taps, int D, std::vector<double>* coef) {
  const int N = D + 1;
  coef->assign((size_t)taps * N, 0.0);
  double fmax = 0.0, emax = 0.0;
  const double ck = c * K;
  for (int t = 0; t < taps; ++t) {
    auto f = [&](double x) { return kb_phi_host((ck - 0.5 + 0.5 * x - t) / c, K, a); };
    std::vector<double> fx(N), ch(N, 0.0);
    for (int k = 0; k < N; ++k) fx[k] = f(std::cos(kPi * (k + 0.5) / N));
    for (int n = 0; n < N; ++n) {
      double acc = 0.0;
      for (int k = 0; k < N; ++k) acc += fx[k] * std::cos(kPi * n * (k + 0.5) / N);
      ch[n] = (n == 0 ? 1.0 : 2.0) * acc / N;
    }
    // Chebyshev -> monomial: T0 = 1, T1 = x, T_{n+1} = 2 x T_n - T_{n-1}
    std::vector<double> tp(N, 0.0), tc(N, 0.0), tn(N, 0.0), mono(N, 0.0);
    tp[0] = 1.0;
    if (N > 1) tc[1] = 1.0;
    for (int i = 0; i < N; ++i) mono[i] += ch[0] * tp[i];
    if (N > 1)
      for (int i = 0; i < N; ++i) mono[i] += ch[1] * tc[i];
    for (int n = 2; n < N; ++n) {
      for (int i = 0; i < N; ++i) tn[i] = (i > 0 ? 2.0 * tc[i - 1] : 0.0) - tp[i];
      for (int i = 0; i < N; ++i) mono[i] += ch[n] * tn[i];
      tp = tc;
      tc = tn;
    }
    for (int i = 0; i < N; ++i) (*coef)[(size_t)t * N + i] = mono[i];
    for (int k = 0; k <= 2000; ++k) {
      const double x = -1.0 + k / 1000.0;
      double p = 0.0;
      for (int i = N - 1; i >= 0; --i) p = p * x + mono[i];
      const double v = f(x);
      fmax = std::fmax(fmax, std::fabs(v));
      emax = std::fmax(emax, std::fabs(p - v));
    }
  }
  return fmax > 0 ? emax / fmax : 0.0;
}

// Gauss-Legendre nodes and weights of order q on [-1, 1]: Newton's method on
// the three-term recurrence of the Legendre polynomials.
void gauss_legendre(int q, std::vector<double>* x, std::vector<double>* w) {
  x->assign(q, 0.0);
  w->assign(q, 0.0);
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = -z;
    (*x)[q - 1 - i] = z;
    (*w)[i] = (*w)[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Cut-off weights of the partial-data model (eq. data-part; w_cut as built at
// the start of Section 5, with the unit-mass bump exp(-1/(1 - |y|^2/eps^2))
// of radius eps convolved with the indicator of the data box shrunk by eps).
// A sample at distance d_i (in steps) from the nearer face of axis i sees the
// part of the bump with y_i <= d_i - eps on that axis (a reflection for an
// upper face; the bump is radial); d_i >= E = ceil(2 eps) leaves the axis
// unconstrained, and 4 eps <= n_i keeps the other face out of reach.  The
// constraint values -eps + j cut [-eps, eps] into E cells per axis; each cell
// of the dim-dimensional grid is integrated by Gauss-Legendre (order q per
// cell piece, about 256 nodes per axis), and prefix sums over the cells give
// W[d1][d2][d3] (index ((d1 (E+1) + d2) (E+1) + d3)), normalised by the
// total.  In 2D the table is over (d1, d3) and repeated along d2.
void cutoff_table(double eps, int dim, std::vector<double>* W) {
  const int E = (int)std::ceil(2.0 * eps - 1e-12);
  const int q = std::max(16, 256 / E);
  std::vector<double> gx, gw;
  gauss_legendre(q, &gx, &gw);
  // nodes and weights of every cell, cell j = [-eps + j, min(-eps + j + 1, eps)]
  std::vector<double> y((size_t)E * q), wy((size_t)E * q);
  for (int j = 0; j < E; ++j) {
    const double a = -eps + j, b = std::min(-eps + j + 1.0, eps), h = 0.5 * (b - a);
    for (int k = 0; k < q; ++k) {
      y[(size_t)j * q + k] = a + h * (gx[k] + 1.0);
      wy[(size_t)j * q + k] = h * gw[k];
    }
  }
  const double ie2 = 1.0 / (eps * eps);
  auto bump = [&](double r2) {
    const double u = 1.0 - r2 * ie2;
    return u > 0.0 ? std::exp(-1.0 / u) : 0.0;
  };
  const int e1 = E + 1;
  W->assign((size_t)e1 * e1 * e1, 0.0);
  if (dim == 3) {
    // cell integrals (symmetric under permutations of the axes)
    std::vector<double> C((size_t)E * E * E, 0.0);
    for (int a = 0; a < E; ++a)
      for (int b = a; b < E; ++b)
        for (int c = b; c < E; ++c) {
          double s = 0.0;
          for (int i = 0; i < q; ++i) {
            const double y1 = y[(size_t)a * q + i], w1 = wy[(size_t)a * q + i];
            for (int j = 0; j < q; ++j) {
              const double y2 = y[(size_t)b * q + j], w12 = w1 * wy[(size_t)b * q + j];
              const double r12 = y1 * y1 + y2 * y2;
              if (r12 >= eps * eps) continue;
              for (int k = 0; k < q; ++k) {
                const double y3 = y[(size_t)c * q + k];
                s += w12 * wy[(size_t)c * q + k] * bump(r12 + y3 * y3);
              }
            }
          }
          const int p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
          for (auto& t : p) C[((size_t)t[0] * E + t[1]) * E + t[2]] = s;
        }
    for (int d1 = 1; d1 <= E; ++d1)
      for (int d2 = 1; d2 <= E; ++d2)
        for (int d3 = 1; d3 <= E; ++d3) {
          auto at = [&](int i, int j, int k) -> double& { return (*W)[((size_t)i * e1 + j) * e1 + k]; };
          at(d1, d2, d3) = C[((size_t)(d1 - 1) * E + (d2 - 1)) * E + (d3 - 1)] + at(d1 - 1, d2, d3) +
                           at(d1, d2 - 1, d3) + at(d1, d2, d3 - 1) - at(d1 - 1, d2 - 1, d3) -
                           at(d1 - 1, d2, d3 - 1) - at(d1, d2 - 1, d3 - 1) + at(d1 - 1, d2 - 1, d3 - 1);
        }
    const double tot = (*W)[((size_t)E * e1 + E) * e1 + E];
    for (double& v : *W) v /= tot;
  } else {
    std::vector<double> C((size_t)E * E, 0.0);
    for (int a = 0; a < E; ++a)
      for (int b = a; b < E; ++b) {
        double s = 0.0;
        for (int i = 0; i < q; ++i)
          for (int j = 0; j < q; ++j) {
            const double y1 = y[(size_t)a * q + i], y2 = y[(size_t)b * q + j];
            s += wy[(size_t)a * q + i] * wy[(size_t)b * q + j] * bump(y1 * y1 + y2 * y2);
          }
        C[(size_t)a * E + b] = C[(size_t)b * E + a] = s;
      }
    std::vector<double> S((size_t)e1 * e1, 0.0);
    for (int d1 = 1; d1 <= E; ++d1)
      for (int d3 = 1; d3 <= E; ++d3)
        S[(size_t)d1 * e1 + d3] = C[(size_t)(d1 - 1) * E + (d3 - 1)] + S[(size_t)(d1 - 1) * e1 + d3] +
                                  S[(size_t)d1 * e1 + d3 - 1] - S[(size_t)(d1 - 1) * e1 + d3 - 1];
    const double tot = S[(size_t)E * e1 + E];
    for (int d1 = 0; d1 <= E; ++d1)
      for (int d2 = 0; d2 <= E; ++d2)
        for (int d3 = 0; d3 <= E; ++d3) (*W)[((size_t)d1 * e1 + d2) * e1 + d3] = S[(size_t)d1 * e1 + d3] / tot;
  }
}

bool is_pow2(int L) { return L > 0 && (L & (L - 1)) == 0; }

int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

bool is_int(double v, double tol = 1e-9) { return std::fabs(v - std::nearbyint(v)) <= tol * std::fmax(1.0, std::fabs(v)); }

template <typename T>
void put(std::vector<unsigned char>& blob, size_t off, const T* v, size_t n) {
  std::memcpy(blob.data() + off, v, n * sizeof(T));
}

}  // namespace

double bessel_i0e(double z) {
  // sum_k (z^2/4)^k / (k!)^2, each term carried with the factor e^{-z} so that
  // nothing overflows for z up to ~700.
  const double q = 0.25 * z * z;
  double term = std::exp(-z);
  double sum = term;
  for (int k = 1; k < 100000; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum && k > z) break;
  }
  return sum;
}

size_t complex_bytes(int prec) { return prec == PAT_F64 ? 16 : 8; }
size_t grid_bytes(int prec) { return prec == PAT_F64 ? 16 : (prec == PAT_F32 ? 8 : 4); }

pat_status build_plan(const pat_geometry& gin, pat_plan* p, std::string* err) {
  std::ostringstream msg;
  auto fail = [&](pat_status s) {
    *err = msg.str();
    return s;
  };
  pat_geometry g = gin;
  if (g.ndim != 2 && g.ndim != 3) {
    msg << "ndim must be 2 or 3 (got " << g.ndim << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  if (g.ndim == 2 && g.nx[1] != 1) {
    msg << "ndim = 2 needs nx[1] = 1 (got " << g.nx[1] << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  for (int a = 0; a < g.ndim - 1; ++a) {
    if (g.nx[a] < 2 || g.nx[a] % 2 != 0) {
      msg << "nx[" << a << "] must be even and >= 2 (got " << g.nx[a] << ")";
      return fail(PAT_ERR_INVALID_ARG);
    }
    if (g.nx[a] > 4096) {
      msg << "nx[" << a << "] = " << g.nx[a] << " exceeds 4096";
      return fail(PAT_ERR_UNSUPPORTED);
    }
  }
  if (g.nt < 2 || g.nt % 2 != 0 || g.nz < 2 || g.nz % 2 != 0) {
    msg << "nt and nz must be even and >= 2 (got " << g.nt << ", " << g.nz << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  if (g.nt > 8192 || g.nz > 8192) {
    msg << "nt, nz above 8192 are not supported";
    return fail(PAT_ERR_UNSUPPORTED);
  }
  if (!finite_pos(g.dx) || !finite_pos(g.dt) || !finite_pos(g.dz) || !finite_pos(g.vs)) {
    msg << "dx, dt, dz, vs must be finite and > 0";
    return fail(PAT_ERR_INVALID_ARG);
  }
  if (g.precision < PAT_F64 || g.precision > PAT_F32_BF16GRID) {
    msg << "unknown precision " << g.precision;
    return fail(PAT_ERR_INVALID_ARG);
  }
  if (g.interp < PAT_INTERP_KB || g.interp > PAT_INTERP_NEAREST) {
    msg << "unknown interp " << g.interp;
    return fail(PAT_ERR_INVALID_ARG);
  }
  {
    const double e = g.cutoff;
    const int n2c = g.ndim == 3 ? g.nx[1] : g.nt;
    if (!std::isfinite(e) || e < 0.0 || e > kMaxCutoff) {
      msg << "cutoff must be 0 or in (0, " << kMaxCutoff << "] sampling steps (got " << e << ")";
      return fail(PAT_ERR_INVALID_ARG);
    }
    if (e > 0.0 && (4.0 * e > g.nx[0] || 4.0 * e > n2c || 4.0 * e > g.nt)) {
      msg << "cutoff " << e << " needs 4 eps <= every data axis length";
      return fail(PAT_ERR_INVALID_ARG);
    }
  }
  const bool kb = g.interp == PAT_INTERP_KB;
  if (!std::isfinite(g.c) || (kb ? g.c <= 1.0 : g.c < 1.0)) {
    msg << "oversampling c must be " << (kb ? "> 1" : ">= 1") << " (got " << g.c << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  // the interpolation-based methods: 2 taps (linear) or 1 (nearest), written
  // as a window of 2cK grid points
  if (g.interp == PAT_INTERP_LINEAR) g.K = 1.0 / g.c;
  if (g.interp == PAT_INTERP_NEAREST) g.K = 0.5 / g.c;
  const double mreal = g.c * g.nt;
  if (!is_int(mreal) || ((long long)std::nearbyint(mreal)) % 2 != 0) {
    msg << "c*nt must be an even integer (got " << mreal << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  const int m = (int)std::nearbyint(mreal);
  if (!std::isfinite(g.K) || g.K <= 0.0) {
    msg << "K must be > 0";
    return fail(PAT_ERR_INVALID_ARG);
  }
  const double tr = 2.0 * g.c * g.K;
  const int min_taps = kb ? 2 : 1;
  if (!is_int(tr) || std::nearbyint(tr) < min_taps || std::nearbyint(tr) > kMaxTaps) {
    msg << "2cK must be an integer in [" << min_taps << ", " << kMaxTaps << "] (got " << tr << ")";
    return fail(PAT_ERR_INVALID_ARG);
  }
  const int taps = (int)std::nearbyint(tr);
  if (m < taps) {
    msg << "c*nt = " << m << " is smaller than the " << taps << " taps";
    return fail(PAT_ERR_INVALID_ARG);
  }
  const double amax = kPi * (2.0 * g.c - 1.0);
  if (kb) {
    if (g.alpha == 0.0) g.alpha = 0.98 * amax;
    if (!std::isfinite(g.alpha) || !(g.alpha > kPi) || !(g.alpha < amax)) {
      msg << "alpha must satisfy pi < alpha < pi(2c-1) = " << amax << " (got " << g.alpha << ")";
      return fail(PAT_ERR_INVALID_ARG);
    }
    if (g.alpha * g.K > 700.0) {
      msg << "alpha*K = " << g.alpha * g.K << " exceeds 700";
      return fail(PAT_ERR_UNSUPPORTED);
    }
  } else {
    g.alpha = 0.0;  // no window parameter
  }
  const int prec = g.precision;
  const size_t cs = complex_bytes(prec);
  const size_t rs = cs / 2;
  // one grid line with its halo of taps must fit one workgroup's LDS (lines
  // whose twiddle table does not fit beside them read it from memory)
  if (((size_t)m + kMaxTaps) * cs > kLdsMax) {
    msg << "c*nt = " << m << " exceeds the LDS line capacity for this precision";
    return fail(PAT_ERR_UNSUPPORTED);
  }

  const int n1 = g.nx[0];
  const int n2 = g.ndim == 3 ? g.nx[1] : 1;
  // FFT plans for every distinct length
  const int lens[4] = {n1, n2, m, g.nz};
  std::vector<int> uniq;
  for (int L : lens) {
    bool seen = false;
    for (int u : uniq) seen = seen || (u == L);
    if (!seen) uniq.push_back(L);
  }
  std::vector<std::vector<int>> rads(uniq.size());
  for (size_t i = 0; i < uniq.size(); ++i) {
    if (!factorize(uniq[i], &rads[i])) {
      msg << "FFT length " << uniq[i] << " has a prime factor above 23";
      return fail(PAT_ERR_UNSUPPORTED);
    }
  }

  Inst I;
  std::memset(&I, 0, sizeof(I));
  I.n1 = n1;
  I.n2 = n2;
  I.nt = g.nt;
  I.nz = g.nz;
  I.m = m;
  I.h1 = n1 / 2 + 1;
  I.lines = I.h1 * n2;
  I.taps = taps;
  I.cut_e = g.cutoff > 0.0 ? (int)std::ceil(2.0 * g.cutoff - 1e-12) : 0;  // cut-off band, steps
  I.tb = prec == PAT_F64 ? 8 : 16;
  while (I.tb > 1 && std::max(lds_tile_x1(I, cs), lds_tile_x2(I, cs)) > 65536) I.tb /= 2;
  I.pow2 = is_pow2(n1) && is_pow2(n2) && is_pow2(m) && is_pow2(g.nz);
  I.lpw_m = clampi(2048 / m, 1, 16);
  I.twg_m = (size_t)m * (I.lpw_m + 1) * cs > kLdsMax ? 1 : 0;
  I.lpw_z = clampi(2048 / g.nz, 1, 16);
  if (lds_line_z(I, cs) > kLdsMax) {
    msg << "nz = " << g.nz << " exceeds the LDS line capacity for this precision";
    return fail(PAT_ERR_UNSUPPORTED);
  }
  I.lpw_i = clampi(2 * kBlock / g.nz, 1, 16);  // one lane per node pair
  while (I.lpw_i > 1 && lds_interp(I, cs) > 65536) --I.lpw_i;
  I.lpw_f = clampi(2048 / m, 1, 16);
  while (I.lpw_f > 1 && lds_fused2(I, cs) > 65536) --I.lpw_f;
  // the adjoint kernel transforms lpw_a depth lines together (power-of-two
  // builds), then spreads them one by one
  I.lpw_a = I.pow2 ? clampi(m / g.nz, 1, 8) : 1;
  // (down to 32 KB of LDS: five workgroups per compute unit)
  while (I.lpw_a > 1 && lds_fused1(I, cs) > 32 * 1024) I.lpw_a /= 2;
  I.c = g.c;
  I.K = g.K;
  I.alpha = g.alpha;
  I.ck = g.c * g.K;
  const double tv = g.nt * g.dt * g.vs;
  I.a1 = (tv / (n1 * g.dx)) * (tv / (n1 * g.dx));
  I.a2 = g.ndim == 3 ? (tv / (n2 * g.dx)) * (tv / (n2 * g.dx)) : 0.0;
  I.b = (tv / (g.nz * g.dz)) * (tv / (g.nz * g.dz));
  I.wcoef = 2.0 * g.vs * (g.dt / g.dz) * std::sqrt(I.b);
  I.scale = 1.0 / (kPi * g.c * (double)n1 * (double)n2 * (double)g.nz);

  // table layout
  size_t off = align256(sizeof(Inst));
  const size_t off_tw = off;
  std::vector<size_t> tw_at(uniq.size());
  size_t tw_elems = 0;
  for (size_t i = 0; i < uniq.size(); ++i) {
    tw_at[i] = tw_elems;
    tw_elems += uniq[i];
  }
  off = align256(off + tw_elems * cs);
  const size_t off_perm = off;
  std::vector<size_t> perm_at(uniq.size());
  size_t perm_elems = 0;
  for (size_t i = 0; i < uniq.size(); ++i) {
    perm_at[i] = perm_elems;
    perm_elems += uniq[i];
  }
  off = align256(off + perm_elems * sizeof(int32_t));
  const size_t off_sn = off;
  off = align256(off + (size_t)g.nt * rs);
  const int deg = prec == PAT_F64 ? kPolyDegD : kPolyDegF;
  std::vector<double> coef;
  I.kind = g.interp;
  I.centred = (g.interp == PAT_INTERP_KB || g.interp == PAT_INTERP_SINC) ? 1 : 0;
  if (kb) {
    const double fit_err = fit_tap_polys(g.c, g.K, g.alpha, taps, deg, &coef);
    I.poly = fit_err <= (prec == PAT_F64 ? 1e-13 : 5e-8) ? 1 : 0;
  } else {
    I.poly = 0;  // the other methods evaluate their weights directly
  }
  {
    // the bf16 option stores the oversampled grid, so it runs the staged
    // kernels; the fused ones need their LDS within one workgroup's share
    I.fused = (kb && prec != PAT_F32_BF16GRID && lds_fused1(I, cs) <= kLdsMax && lds_fused2(I, cs) <= kLdsMax) ? 1 : 0;
  }
  const size_t off_poly = off;
  off = align256(off + coef.size() * rs);
  std::vector<double> cutw;
  if (I.cut_e) cutoff_table(g.cutoff, g.ndim, &cutw);
  const size_t off_cut = off;
  off = align256(off + cutw.size() * rs);
  const size_t total = off;

  p->blob.assign(total, 0);
  for (size_t i = 0; i < uniq.size(); ++i) {
    const int L = uniq[i];
    for (int k = 0; k < L; ++k) {
      // exp(-2 pi i k / L), argument formed from the reduced fraction k/L
      const double ang = 2.0 * kPi * ((double)k / (double)L);
      const double re = std::cos(ang), im = -std::sin(ang);
      const size_t o = off_tw + (tw_at[i] + k) * cs;
      if (prec == PAT_F64) {
        const double v[2] = {re, im};
        put(p->blob, o, v, 2);
      } else {
        const float v[2] = {(float)re, (float)im};
        put(p->blob, o, v, 2);
      }
    }
    const std::vector<int32_t> pos = dif_positions(L, rads[i]);
    put(p->blob, off_perm + perm_at[i] * sizeof(int32_t), pos.data(), pos.size());
  }
  auto desc_of = [&](int L) {
    FftDesc d;
    std::memset(&d, 0, sizeof(d));
    for (size_t i = 0; i < uniq.size(); ++i) {
      if (uniq[i] == L) {
        d.L = L;
        d.nst = (int)rads[i].size();
        for (size_t s = 0; s < rads[i].size(); ++s) d.rad[s] = rads[i][s];
        d.tw = (int32_t)tw_at[i];
        d.perm = (int32_t)perm_at[i];
      }
    }
    return d;
  };
  I.f1 = desc_of(n1);
  I.f2 = desc_of(n2);
  I.fm = desc_of(m);
  I.fz = desc_of(g.nz);
  // deconvolution factors e^{alpha K} / I0(K sqrt(alpha^2 - theta_n^2)),
  // theta_n = 2 pi n / nt - pi  (eq. nufft-c with Psi the Kaiser-Bessel window)
  // (1 for the other methods: Psi = 1 there, or no window at all)
  for (int n = 0; n < g.nt; ++n) {
    const double th = 2.0 * kPi * ((double)n / (double)g.nt) - kPi;
    const double z = g.K * std::sqrt(g.alpha * g.alpha - th * th);
    const double s = kb ? std::exp(g.alpha * g.K - z) / bessel_i0e(z) : 1.0;
    const size_t o = off_sn + (size_t)n * rs;
    if (prec == PAT_F64) {
      put(p->blob, o, &s, 1);
    } else {
      const float f = (float)s;
      put(p->blob, o, &f, 1);
    }
  }
  for (size_t i = 0; i < cutw.size(); ++i) {
    const size_t o = off_cut + i * rs;
    if (prec == PAT_F64) {
      put(p->blob, o, &cutw[i], 1);
    } else {
      const float f = (float)cutw[i];
      put(p->blob, o, &f, 1);
    }
  }
  for (size_t i = 0; i < coef.size(); ++i) {
    const size_t o = off_poly + i * rs;
    if (prec == PAT_F64) {
      put(p->blob, o, &coef[i], 1);
    } else {
      const float f = (float)coef[i];
      put(p->blob, o, &f, 1);
    }
  }
  // workspace: G (lines x nt), grid (lines x m), F (lines x nz)
  const size_t lines = (size_t)I.lines;
  I.off_g = 0;
  I.off_u = (int64_t)align256(lines * g.nt * cs);
  I.off_f = I.off_u + (int64_t)align256(lines * (size_t)m * grid_bytes(prec));
  p->ws_bytes = (size_t)I.off_f + align256(lines * g.nz * cs);

  p->g = g;
  p->prec = prec;
  p->fusable = I.fused != 0;
  p->spread_ok = lds_spread(I, complex_bytes(prec)) <= kLdsMax;
  p->inst = I;
  p->off_desc = 0;
  p->off_tw = off_tw;
  p->off_perm = off_perm;
  p->off_sn = off_sn;
  p->off_poly = off_poly;
  p->off_cut = off_cut;
  p->table_bytes = total;
  return PAT_OK;
}

void bind_table(pat_plan* p, void* table_dev) {
  unsigned char* base = static_cast<unsigned char*>(table_dev);
  p->inst.tw = base + p->off_tw;
  p->inst.perm = reinterpret_cast<const int32_t*>(base + p->off_perm);
  p->inst.sn = base + p->off_sn;
  p->inst.poly_c = base + p->off_poly;
  p->inst.cutw = p->inst.cut_e ? base + p->off_cut : nullptr;
  std::memcpy(p->blob.data() + p->off_desc, &p->inst, sizeof(Inst));
  p->table_dev = table_dev;
}

}  // namespace pat
