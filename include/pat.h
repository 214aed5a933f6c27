/*
 * pat.h - C ABI of libpatnufft: NUFFT-based Fourier reconstruction for
 * photoacoustic imaging with a planar (3D) or line (2D) detector array.
 *
 * The operation is the partial Fourier reconstruction f^dagger of the paper's
 * Section 2 (eq. inv2), discretised as in Section 4 (eqs. gd, fd, dft-2d,
 * fft-1a, fft-2, fft-0, fft-1) and evaluated with the one-dimensional
 * nonuniform FFT of Section 3 (Proposition on the NUFFT identity, eqs.
 * nufft-a / nufft-c, the NUFFT algorithm, Kaiser-Bessel window of Section
 * 3.2): detector data p(x, t) in, initial pressure f(x, z) out.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays are C-contiguous.  Detector data p has shape (nx[0], nx[1], nt)
 *    with time fastest; images f have shape (nx[0], nx[1], nz) with depth
 *    fastest.  The 2D line-detector geometry uses ndim = 2 and nx[1] = 1.
 *  - Detector m sits at x = m*dx on the plane y = 0, sample n at t = n*dt,
 *    image sample q at depth y = q*dz (Section 4 discretisation).
 *  - Element type: double for PAT_F64, float for PAT_F32 and
 *    PAT_F32_BF16GRID (the latter stores only the oversampled grid in bf16).
 *  - Every device pointer is caller-owned device memory on the device that is
 *    current when the call is made, 16-byte aligned, and comes with its size
 *    in bytes.  The library allocates no device memory: the plan's constant
 *    tables live in a caller buffer of pat_plan_sizes().table_bytes filled by
 *    pat_plan_upload(), and every transform takes a caller workspace of
 *    pat_plan_sizes().workspace_bytes.  A table or workspace smaller than that
 *    gives PAT_ERR_WORKSPACE, an array smaller than its shape needs
 *    PAT_ERR_INVALID_ARG.  Array sizes: data p  nx[0] nx[1] nt  elements,
 *    image f  nx[0] nx[1] nz  elements (double for PAT_F64, else float);
 *    line-stage arrays as described at pat_nufft2_lines.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work; results are ready when the stream is.
 *  - Errors: every argument is validated before anything is enqueued, so a
 *    non-OK status means nothing was written.  A HIP launch failure reports
 *    PAT_ERR_HIP; an asynchronous fault of earlier work surfaces on a later
 *    HIP call.  pat_last_error() gives a thread-local message for the last
 *    non-OK status.  No C++ exception crosses this boundary.
 *  - A plan may be used from one host thread at a time; different plans are
 *    independent.  Calls that share a workspace must be stream-ordered.
 *  - Error injection: the environment variable PAT_FAULT, read at every call
 *    that would touch the GPU, makes one HIP step report a failure before it
 *    runs, so that the PAT_ERR_HIP path can be exercised: "upload" (the table
 *    copy of pat_plan_upload), "scratch" (the scratch lookup of
 *    pat_reconstruct_noalloc), "launch" or "launch:k" (the k-th kernel launch
 *    of the operator, k >= 1; the kernels before it run, the output array is
 *    written by the last kernel only and stays untouched).  Unset or empty:
 *    no effect.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAT_OK = 0,
  PAT_ERR_INVALID_ARG = 1, /* null/misaligned pointer, bad geometry value */
  PAT_ERR_UNSUPPORTED = 2, /* valid but outside what the library supports */
  PAT_ERR_WORKSPACE = 3,   /* table not uploaded / workspace missing */
  PAT_ERR_HIP = 4,         /* a HIP runtime call failed */
  PAT_ERR_INTERNAL = 5
} pat_status;

typedef enum {
  PAT_F64 = 0,          /* every stage in double */
  PAT_F32 = 1,          /* float; node, phase, weight and deconvolution
                           factors formed in double */
  PAT_F32_BF16GRID = 2  /* as PAT_F32, oversampled grid stored as bf16 */
} pat_precision;

/* How the nonuniform sums of eq. (fft-2) are evaluated (Section 4 compares
 * these).  PAT_INTERP_KB is the NUFFT-based algorithm (Section 3) and the only
 * one every entry point supports; the others serve the accuracy-against-time
 * comparison and run pat_reconstruct and pat_nufft2_lines only (staged
 * kernels), the remaining operators returning PAT_ERR_UNSUPPORTED:
 *  SINC     the NUFFT algorithm with Psi = 1 on [-c pi, c pi] ("truncated
 *           sinc"): no deconvolution, 2cK taps of sin(c pi u)/u.
 *  LINEAR   interpolation-based: the zero-padded FFT at omega = j/c, linear
 *           interpolation between floor(c omega) and the next grid point
 *           (K and alpha are ignored; c >= 1).
 *  NEAREST  as LINEAR with the nearest grid point, floor(c omega + 1/2). */
typedef enum {
  PAT_INTERP_KB = 0,
  PAT_INTERP_SINC = 1,
  PAT_INTERP_LINEAR = 2,
  PAT_INTERP_NEAREST = 3
} pat_interp;

/*
 * Geometry and NUFFT parameters.
 *  ndim      2 (line detectors, nx[1] must be 1) or 3 (planar array).
 *  nx[0..1]  detectors per transverse axis; even (nx[1] = 1 allowed in 2D),
 *            2 <= nx <= 4096.
 *  nt, nz    time samples and output depth samples; even, 2 <= . <= 8192.
 *  dx,dt,dz  detector spacing, time step, depth spacing (> 0).
 *  vs        speed of sound (> 0).
 *  c         oversampling factor of the NUFFT (Section 3.1, eq. nufft-c),
 *            c > 1 with c*nt an even integer.
 *  K         interpolation length (Section 3.1 step (ii)); 2*c*K must be an
 *            integer between 2 and 64 (the number of taps per node).
 *  alpha     Kaiser-Bessel width (Section 3.2), pi < alpha < pi*(2c-1);
 *            0 selects 0.98*pi*(2c-1), just below the upper limit, as the
 *            numerical experiments of Section 5 do.
 *  precision a pat_precision.
 *  interp    a pat_interp value; PAT_INTERP_KB, the Kaiser-Bessel NUFFT, is
 *            the method of the paper.
 *  cutoff    radius eps, in sampling steps, of the smooth cut-off w_cut of
 *            the partial-data model (eq. data-part; its construction at the
 *            start of Section 5); 0 disables it (w = 1).  w_cut is the bump
 *            exp(-1/(1 - |y|^2/eps^2)) of radius eps and unit mass, convolved
 *            with the indicator of the data box shrunk by eps, in the
 *            coordinates (x1, x2, t) (2D: (x1, t)) measured in sampling
 *            steps, with data sample s of an axis of n samples at s and the
 *            data box [0, n]: w is 0 on the box faces, 1 from 2 eps inwards,
 *            smooth between.  The operators then act on w p: R(w p),
 *            w R^T(q), w A(f), A^T(w p).  0 < eps <= 8 and 4 eps <= every
 *            data axis length (n1, n2 in 3D, nt), else PAT_ERR_INVALID_ARG.
 * Every FFT length (nx[0], nx[1], nz, c*nt) must factor into primes <= 23.
 * A line of c*nt complex values with a halo of 64 taps must fit one
 * workgroup's LDS (160 KB): c*nt <= 20416 in float, 10176 in double (16384
 * and 8192 among the powers of two); the fused line kernels hold a line
 * twice, plus per-node lists, so about half of that (c*nt = 8192 in float
 * and 4096 in double fit; larger plans run the staged kernels, and
 * pat_plan_set_fused(plan, 1) returns PAT_ERR_UNSUPPORTED for them).  A
 * depth line pair (2 nz values) must fit as well, nz <= 5120 in double.
 * Larger sizes make pat_plan_create return PAT_ERR_UNSUPPORTED.  The
 * operators that spread (reconstruct adjoint, forward model, nufft1_lines)
 * also keep per-node lists of a depth line in LDS, (nz + 2) * (8 + 4 + 4 r)
 * bytes in float and (nz + 2) * (16 + 4 + 8 r) in double with r = (2cK + 6)
 * | 1: nz up to about 1800 (float) and 900 (double) at 12 taps; beyond that
 * those calls return PAT_ERR_UNSUPPORTED.
 */
typedef struct {
  int32_t ndim;
  int32_t nx[2];
  int32_t nt, nz;
  double dx, dt, dz, vs;
  double c, K, alpha;
  int32_t precision;
  int32_t interp;
  double cutoff;
} pat_geometry;

typedef struct pat_plan pat_plan;

/* Host-only: validates the geometry and builds the FP64 constant tables
 * (deconvolution factors 1/Psi(2 pi n/nt - pi), FFT twiddles, index maps).
 * Never touches the GPU.  *out receives a new plan, freed by
 * pat_plan_destroy(). */
pat_status pat_plan_create(const pat_geometry* geom, pat_plan** out);

/* Bytes of the device table buffer and of the workspace every transform of
 * this plan needs.  Either output pointer may be NULL. */
pat_status pat_plan_sizes(const pat_plan* plan, size_t* table_bytes, size_t* workspace_bytes);

/* Copies the plan's tables into table_dev (table_bytes, caller-owned, must
 * stay alive while the plan is used) on `stream`, then synchronises the
 * stream.  Must precede any transform. */
pat_status pat_plan_upload(pat_plan* plan, void* table_dev, size_t table_bytes, void* stream);

/* R: reconstruction (Section 4, the NUFFT-based algorithm).  p -> f.
 *   a1  DFT over the detector axes (eq. fft-1a),
 *   a2  deconvolution by 1/Psi, zero padding to c*nt, FFT (eq. nufft-c),
 *   a3  2cK-tap Kaiser-Bessel interpolation at the nodes
 *       nu_{k,l} = sign(l) nt dt vs |K| / (2 pi) (eqs. nufft-a, dft-2d),
 *       times the Jacobian weight 2 vs (dt/dz) |K_z| / |K| (eqs. fft-0, inv),
 *   a4, a5  inverse DFT over depth and detector axes, real part (eq. fft-1).
 * The weight is 0 on the plane l = 0; on the depth-Nyquist plane l = -nz/2
 * the value is the mean of the two nodes +-|nu| (the real part of eq. fft-1).
 * p, f: device arrays as described above.  ws: workspace_bytes. */
pat_status pat_reconstruct(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes, void* ws,
                           size_t ws_bytes, void* stream);

/* R as pat_reconstruct, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument, and the call allocates nothing.  Its
 * workspace is a static array of the library, 64 MiB per device, reserved
 * when the library's code is first loaded on that device and held until the
 * process ends; its address is looked up once per device.  The fused line
 * path needs lines*(nt + nz) complex elements of it (256-byte aligned parts),
 * the staged path pat_plan_sizes().workspace_bytes; a plan needing more gets
 * PAT_ERR_UNSUPPORTED before anything is enqueued (FP32 fits up to about
 * 128^2 x 256 -> 128^3; 256^2 x 512 does not).  Every call on a device shares
 * that device's array and leaves its contents behind (nothing in it needs
 * clearing: each call writes every part it reads).  Calls that overlap on one
 * device, on different streams or host threads, race on the array and must
 * be serialised by the caller.  Results equal pat_reconstruct's. */
pat_status pat_reconstruct_noalloc(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes,
                                   void* stream);

/* R^T: the exact transpose of R for the real inner product (type-1 NUFFT
 * spreading; the gradient of R).  f-shaped input -> p-shaped output. */
pat_status pat_reconstruct_adjoint(pat_plan* plan, const void* f, size_t f_bytes, void* p, size_t p_bytes,
                                   void* ws, size_t ws_bytes, void* stream);

/* A: the spectral forward model of the wave problem of Section 2 on the
 * periodic sampling grid, p[m, n] = Re( IDFT_x( (1/nz) sum_l F[k, l]
 * cos(2 pi |nu_{k,l}| n / nt) ) ), F the DFT of f over all axes; evaluated as
 * a type-1 NUFFT (spreading to the nodes +-|nu|).  f -> p. */
pat_status pat_forward(pat_plan* plan, const void* f, size_t f_bytes, void* p, size_t p_bytes, void* ws,
                       size_t ws_bytes, void* stream);

/* A^T: transpose of A (type-2 interpolation at +-|nu|).  p -> f-shaped. */
pat_status pat_forward_adjoint(pat_plan* plan, const void* p, size_t p_bytes, void* f, size_t f_bytes, void* ws,
                               size_t ws_bytes, void* stream);

/* R for n independent plans (1 <= n <= 32).  The plans are grouped by the
 * radix class of their FFT lengths (the butterflies a kernel build carries);
 * each group runs one launch per stage, whose persistent grid draws work
 * items (instance, tile or line) from a device work counter.  The first group
 * runs on `stream`; the others run on two streams of plans[0]'s own (created
 * on its first batched call with the default priority, released by
 * pat_plan_destroy), forked from `stream` after the work counters are
 * cleared and joined back into it before the call returns, so that work the
 * caller enqueues on `stream` afterwards sees every output.  With timing on
 * (pat_plan_set_timing on plans[0]) everything runs on `stream`.  All plans
 * must share one precision.  p[i], f[i] as for pat_reconstruct of plans[i];
 * ws of pat_batched_workspace_size() bytes.  If a launch fails, each f[i] is
 * either complete or untouched. */
pat_status pat_batched_workspace_size(int32_t n, pat_plan* const* plans, size_t* workspace_bytes);
pat_status pat_reconstruct_batched(int32_t n, pat_plan* const* plans, const void* const* p,
                                   const size_t* p_bytes, void* const* f, const size_t* f_bytes, void* ws,
                                   size_t ws_bytes, void* stream);

/* Stage a3 alone (type-2 interpolation + weight) on the half spectrum.
 * grid: (lines, c*nt) complex, lines = (nx[0]/2+1)*nx[1], line (k1, k2) at
 *   row k1*nx[1] + k2 (k2 in DFT order), interleaved (re, im) in the plan's
 *   grid storage (double, float or bf16 pairs).  Row j of a line holding the
 *   detector-DFT values G[n] is what stage a2 writes (eq. nufft-c, centred):
 *     U[j] = sum_n G[n] e^{alpha K} / (I0(alpha K) Psi(2 pi n/nt - pi))
 *                   * exp(-2 pi i j (n - nt/2) / (c nt)).
 * out: (lines, nz) complex in the plan's element type, l in DFT order:
 *   W_{k,l} T[G](nu_{k,l}) / (nx[0] nx[1] nz), with the l = 0 and l = -nz/2
 *   conventions of pat_reconstruct. */
pat_status pat_nufft2_lines(pat_plan* plan, const void* grid, size_t grid_bytes, void* out, size_t out_bytes,
                            void* stream);

/* Spreading alone (type-1; the step of R^T that pat_nufft2_lines mirrors):
 * the exact adjoint of pat_nufft2_lines for the complex inner product,
 *   grid = N^H values  where  out = N grid  is pat_nufft2_lines,
 * so every grid cell gathers the 2cK-tap kernel weights of the nodes whose
 * window covers it (periodic in the grid index), times conj(W e^{-i pi nu})
 * / (nx[0] nx[1] nz); on l = -nz/2 the value feeds both nodes -+|nu| with
 * half weight.  values: (lines, nz) complex in the plan's element type, l in
 * DFT order; grid: (lines, c*nt) in the plan's grid storage.  Deterministic
 * (no atomics). */
pat_status pat_nufft1_lines(pat_plan* plan, const void* values, size_t values_bytes, void* grid,
                            size_t grid_bytes, void* stream);

/* Line-stage layout.  By default (fused = 1) the deconvolution, oversampled
 * FFT, interpolation and depth DFT of each line group run in one kernel and
 * the oversampled grid never reaches memory (likewise for the spreading
 * side).  fused = 0 runs them as separate kernels that store the grid in the
 * workspace.  PAT_F32_BF16GRID plans are always staged (the option concerns
 * the stored grid): asking them for fused = 1 returns PAT_ERR_UNSUPPORTED. */
pat_status pat_plan_set_fused(pat_plan* plan, int32_t fused);

/* Per-kernel timing.  pat_plan_set_timing(plan, 1) makes later transforms of
 * this plan (and batched calls whose first plan it is) record a hipEvent
 * before and after every kernel on their stream.  pat_plan_stage_times()
 * synchronises on those events, writes up to `cap` records in launch order
 * (names[i]: static strings, ms[i]: kernel time) and the number of records
 * through *count, then forgets them; records accumulate until then. */
pat_status pat_plan_set_timing(pat_plan* plan, int32_t on);
pat_status pat_plan_stage_times(pat_plan* plan, int32_t cap, const char** names, float* ms,
                                int32_t* count);

void pat_plan_destroy(pat_plan* plan);
const char* pat_status_string(pat_status s);
const char* pat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PAT_H */
