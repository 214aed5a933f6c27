// Internal data shared by the host plan (plan.cpp), the kernels
// (kernels.hip) and the C ABI layer (capi.cpp).  Plain structs only: the
// descriptor is built on the host in FP64 and copied verbatim to the device.
#pragma once

#include <cstddef>
#include <cstdint>

namespace pat {

constexpr int kMaxStages = 16;   // radix stages of one FFT
constexpr int kMaxBatch = 32;    // instances in one batched call
constexpr int kMaxTaps = 64;     // 2cK
constexpr double kMaxCutoff = 8.0;  // cut-off radius in sampling steps
constexpr int kBlock = 256;      // threads per workgroup of every kernel
constexpr int kNumCounters = 32; // persistent work counters per batched call (8 per radix class)
// Bytes of the static per-device scratch array behind the allocation-free
// entry point (pat_reconstruct_noalloc); a plan whose workspace needs more is
// refused there.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;   // devices the scratch addresses are cached for
constexpr size_t kLdsMax = 160 * 1024;  // LDS of one CDNA4 compute unit
constexpr double kPi = 3.14159265358979323846264338327950288;
// Degree of the per-tap polynomial that replaces the kernel evaluation
// (float and double paths).
constexpr int kPolyDegF = 8;
constexpr int kPolyDegD = 15;
// 32-bit words of the mirrored tap-pair coefficients passed in kernel arguments
constexpr int kPolyWords = 192;

// One FFT length: in-place decimation-in-frequency mixed-radix factorisation.
// After the transform the natural-order bin k sits at LDS position perm[k].
struct FftDesc {
  int32_t L;
  int32_t nst;
  int32_t rad[kMaxStages];
  int32_t tw;    // element offset of the L roots exp(-2 pi i k / L) in the twiddle table
  int32_t perm;  // element offset of the bin -> position map in the index table
};

// Everything a kernel needs about one reconstruction instance.
struct Inst {
  int32_t n1, n2, nt, nz, m;  // detectors, time samples, depth samples, c*nt
  int32_t h1;                 // n1/2 + 1 (half spectrum over the first axis)
  int32_t lines;              // h1 * n2 frequency lines
  int32_t taps;               // 2cK
  int32_t tb;                 // batch width of the transverse tiles
  int32_t poly;               // 1: per-tap polynomial table valid, 0: direct kernel evaluation
  int32_t lpw_m, lpw_z, lpw_i;  // lines per work item: length-m FFT stages, depth FFT, interp/spread
  int32_t pow2;               // every FFT length is a power of two
  int32_t lpw_f;              // lines per work item of the fused line kernels
  int32_t lpw_a;              // lines per work item of the fused adjoint kernel
  int32_t kind;               // pat_interp: how the nonuniform sums are evaluated
  int32_t centred;            // grid from centred samples (KB, sinc) or not (linear, nearest)
  int32_t fused;              // 1: line stages fused in LDS (grid never stored), 0: staged
  int32_t cut_e;              // cut-off band width E = ceil(2 eps) in samples; 0: no cut-off
  int32_t twg_m;              // 1: the staged grid-line kernels read the c*nt-point twiddles from
                              // memory (table and line together exceed LDS), 0: from LDS
  double c, K, alpha;
  double ck;                  // c*K
  // node and weight:  nu+^2 = a1 k1^2 + a2 k2^2 + b l^2 ;  W = wcoef |l| / nu+
  double a1, a2, b, wcoef;
  // 1 / (pi c n1 n2 nz): the 1/(2 pi c) of the NUFFT identity with the factor
  // 2 e^{alpha K} folded into the deconvolution table, and the inverse-DFT
  // normalisation.
  double scale;
  FftDesc f1, f2, fm, fz;
  // device addresses inside this instance's table buffer (set at upload)
  const void* tw;        // cplx<T>[]
  const int32_t* perm;   // int32[]
  const void* sn;        // T[nt]: e^{alpha K} / I0(K sqrt(alpha^2 - theta_n^2))
  const void* poly_c;    // T[taps][deg+1]: tap t as a polynomial in x = 2 (delta - cK) + 1
  // T[(E+1)^3]: cut-off weight by the samples' distances d_i = min(s, n - s)
  // to the data box faces per axis (x1, x2, t), each clamped to E; entry
  // ((d1 (E+1) + d2) (E+1) + d3).  2D plans use d2 = E.
  const void* cutw;
  // workspace byte offsets
  int64_t off_g, off_u, off_f;
};

// LDS bytes each kernel needs for one instance (cs: bytes per complex
// element, rs: per real).  The kernels carve their LDS exactly as described
// here; the host plan uses the same functions for its capacity checks and the
// launchers for the dynamic LDS request.
// (FFT kernels start with the twiddle table of each length they transform)
// (x1 passes: plus one column's (E+1)^2 cut-off weights when a cut-off is set)
inline size_t lds_tile_x1(const Inst& I, size_t cs) {
  const size_t e1 = (size_t)I.cut_e + 1;
  return (size_t)I.n1 * (I.tb + 1) * cs + (I.cut_e ? e1 * e1 * (cs / 2) : 0);
}
inline size_t lds_tile_x2(const Inst& I, size_t cs) { return (size_t)I.n2 * (I.tb + 1) * cs; }
inline size_t lds_line_z(const Inst& I, size_t cs) { return (size_t)I.nz * (I.lpw_z + 1) * cs; }
inline size_t lds_line_m(const Inst& I, size_t cs) { return (size_t)I.m * (I.lpw_m + (I.twg_m ? 0 : 1)) * cs; }
// interp: lpw_i grid lines of m entries plus a halo of taps - 1
inline size_t lds_interp(const Inst& I, size_t cs) { return (size_t)I.lpw_i * ((size_t)I.m + I.taps) * cs; }
// streamed interp: one buffer of lpw_i lines, line stride m + taps - 1
// rounded up to 16 bytes
inline size_t lds_interp_stream(const Inst& I, size_t cs) {
  const size_t q = cs >= 16 ? 1 : 16 / cs;
  const size_t ls = ((size_t)I.m + I.taps - 1 + q - 1) / q * q;
  return (size_t)I.lpw_i * ls * cs;
}
// spreading lists: per-node value, zero-padded tap-weight row (taps + 6
// entries, made odd), first tap; nz + 2 nodes at most
inline size_t lds_spread_lists(int nz, int taps, size_t cs, int kcells = 4) {
  const size_t row = (size_t)((taps + 2 * (kcells - 1)) | 1);
  return ((size_t)nz + 2) * (cs + row * (cs / 2) + sizeof(int32_t));
}
// stand-alone spreading gathers 4 cells per thread, the fused adjoint 2
inline size_t lds_spread(const Inst& I, size_t cs) { return lds_spread_lists(I.nz, I.taps, cs); }
inline size_t lds_spread_fused(const Inst& I, size_t cs) { return lds_spread_lists(I.nz, I.taps, cs, 2); }
// fused type-2 line kernel: lpw_f lines of max(m, nz) (FFT scratch, then the
// depth line) and lpw_f grid lines of m (natural order, no halo: at 1024
// points two lines take exactly 32 KB, five workgroups per compute unit)
inline size_t lds_fused2(const Inst& I, size_t cs) {
  const size_t sp = (size_t)(I.m > I.nz ? I.m : I.nz);
  return (size_t)I.lpw_f * (sp + (size_t)I.m) * cs;
}
// FP32 spreading by wavefronts: one grid line of m complex floats per
// wavefront of the workgroup (stand-alone), plus the depth spectra in the
// fused type-1 kernel
inline size_t lds_spread_wave(const Inst& I) { return (size_t)(kBlock / 64) * I.m * 8; }
inline size_t lds_fused1_wave(const Inst& I, size_t cs) {
  return (size_t)(kBlock / 64) * ((size_t)I.m + I.nz) * cs;
}
// fused type-1 line kernel: a region of max(m, lpw_a nz) (the depth FFTs,
// then one grid line), lpw_a depth spectra in natural order, the lists
inline size_t lds_fused1(const Inst& I, size_t cs) {
  const size_t za = (size_t)I.lpw_a * I.nz;
  return ((size_t)I.m > za ? (size_t)I.m : za) * cs + za * cs + lds_spread_fused(I, cs);
}

}  // namespace pat
