/*
 * pencilfft.h -- C ABI of the MI355X (gfx950) pencil 3D real-to-complex /
 * complex-to-real FFT library.
 *
 * The method is the transpose-based 3D FFT of Pekurovsky, "P3DFFT: a
 * framework for parallel computations of Fourier transforms in three
 * dimensions" (arXiv:1905.02803): three stages of batched 1D transforms, along
 * X (real-to-complex), then Y, then Z (complex-to-complex), with the data
 * re-oriented from X-pencils to Y-pencils to Z-pencils between stages
 * (Sec. 2, Fig. 2).  The backward transform runs the chain in reverse, ending
 * in a complex-to-real transform along X (Sec. 3.2).  On one GPU the paper's
 * pack / all-to-all / unpack steps (Sec. 3.3) become on-device reorders fused
 * into the transform kernels' loads and stores.
 *
 * Conventions (Sec. 3.2, Table 1, Sec. 4.1):
 *  - Arrays are C order, slowest index first.  The paper's Fortran storage
 *    order "XYZ" (X fastest) is C [z][y][x].
 *  - Real X-pencil data: float or double [nz][ny][nx], unpadded.
 *  - Half spectrum: nxh = nx/2 + 1 complex modes along X (the paper's
 *    (Nx+2)/2 in integer division; modes above nx/2 follow by conjugate
 *    symmetry).  Complex values are interleaved (re, im) pairs of the plan's
 *    precision.
 *  - Z-pencil complex data: with stride1 = 1 (the paper's "STRIDE1 defined",
 *    Fortran ZYX) C [nxh][ny][nz] (kz fastest); with stride1 = 0 (Fortran XYZ)
 *    C [nz][ny][nxh].
 *  - Forward uses exp(-2 pi i ...), backward exp(+2 pi i ...); neither is
 *    normalised, so backward(forward(u)) = nx*ny*nz * u (Sec. 4.1: the round
 *    trip returns the input up to a scale factor).
 *  - Backward is the staged transform: inverse C2C along Z, then along Y, then
 *    along X the 1D C2R that uses only the real parts of mode 0 and (even nx)
 *    mode nx/2, the two modes Sec. 3.2 states are real.  On any output of the
 *    forward transform this is the inverse 3D DFT.
 *
 * Ownership and ordering: the caller owns every data buffer (device memory);
 * the plan owns its twiddle tables and, unless pf_set_workspace supplied one,
 * its workspace.  Transform calls only enqueue work on the given stream
 * (a hipStream_t; NULL means the default stream) and return at once.  A plan
 * must not be used from two streams concurrently: its workspace is shared.
 *
 * Errors: every call returns PF_OK (0) or a negative PF_E* code; nothing is
 * thrown across the ABI.  pf_strerror names a code.
 */
#ifndef PENCILFFT_H
#define PENCILFFT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PF_OK 0
#define PF_EINVAL (-1)        /* bad sizes, layout values or arguments        */
#define PF_EUNSUPPORTED (-2)  /* length with a prime factor above 7, option
                                 not built, or math/precision combination     */
#define PF_EALIGN (-3)        /* data pointer not 16-byte aligned             */
#define PF_EALIAS (-4)        /* in == out but the plan is out-of-place, or
                                 in != out but the plan is in-place           */
#define PF_ENOMEM (-5)        /* device allocation failed                     */
#define PF_EWORKSPACE (-6)    /* workspace missing or too small               */
#define PF_EHIP (-7)          /* a HIP runtime call or kernel launch failed   */
#define PF_ETIMEOUT (-8)      /* a fused pass's bounded wait expired (pf_check_status) */

/* ---- layout option values ---------------------------------------------- */
#define PF_F32 0 /* single precision (Sec. 3.1: single and double supported) */
#define PF_F64 1

/*
 * math: PF_PLAIN computes every butterfly on the vector ALUs in the plan
 * precision.  The MFMA options (F32 plans only) run both radix-16 stages of
 * the power-of-two passes (lengths 512 and 1024 for Y and Z, nx 1024 and 2048
 * for X, i.e. 16 x 16 x R with R = 2 or 4) as 16 x 16 complex DFT-matrix
 * products on the matrix cores, with both operands split into high and low
 * half-precision parts (three products, FP32 accumulation); FP16 inputs are
 * scaled by a power of two per butterfly; twiddles and the last radix-R stage
 * stay FP32 on the vector ALUs.  The first stage reads its operands straight
 * from the loaded registers (where the input side is 16-byte aligned rows or
 * lines; a Z pass reading unaligned [nz][ny][nxh] rows keeps it on the
 * vector ALUs).  Other passes run as PF_PLAIN.  The result differs from
 * PF_PLAIN by rounding only: FP16 x 2 is FP32-class, BF16 x 2 has an error
 * floor of about 2^-16 per product (relative L2 against the FP64 oracle is
 * reported by the tests).
 */
#define PF_PLAIN 0
#define PF_MFMA_FP16X2 1
#define PF_MFMA_BF16X2 2

#define PF_THIRD_FFT 0   /* Fourier transform along Z (default)                 */
#define PF_THIRD_EMPTY 1 /* no transform along Z (Sec. 3.1: empty transform)   */
#define PF_THIRD_CHEB 2  /* type-I DCT along Z on nz Gauss-Lobatto points     */
                         /* (Sec. 3.1: Chebyshev third transform), unnormalised */

#define PF_PENCIL_X 0
#define PF_PENCIL_Y 1
#define PF_PENCIL_Z 2

#define PF_DIR_FORWARD 0
#define PF_DIR_BACKWARD 1

/*
 * Layout and options of a plan.  Initialise with pf_layout_init, then change
 * fields.  m1 x m2 is the virtual processor grid of Sec. 2 (m1 * m2 = P; 1 x P
 * is the slab decomposition of Sec. 4.3); the default 1 x 1 is one whole grid.
 * With m1 * m2 > 1 the user arrays are the P ranks' local pencil blocks of
 * Table 1, concatenated in rank order r2 * m1 + r1, each block in its Table 1
 * storage order (pf_query_dims gives each block's extents): the forward input
 * is the ranks' X-pencils, the forward output their Z-pencils (and the reverse
 * for the backward transform).  The results equal the corresponding slices of
 * the 1 x 1 transform bit for bit.  stride1 selects the Table 1 storage orders
 * (Sec. 3.2, 3.3).  useeven asks for exchange blocks padded to equal size
 * (Sec. 3.4), a property of the message buffers of an all-to-all; on one GPU
 * the exchanges are on-device permutations without message buffers, so the
 * flag is accepted and changes no result and no layout.  third =
 * PF_THIRD_EMPTY skips the transform along Z (Sec. 3.1): the forward output
 * is the Z-pencil of the X-then-Y transformed data, z untransformed, and the
 * backward transform starts from such an array; nz may then have any prime
 * factors (nothing is transformed along z).  third = PF_THIRD_CHEB
 * replaces the Z FFT by the type-I DCT Y[k] = x[0] + (-1)^k x[nz-1] + 2
 * sum_{j=1}^{nz-2} x[j] cos(pi j k / (nz - 1)) in both directions (it is its
 * own inverse up to 2 (nz - 1), so the round trip returns nx ny 2 (nz - 1) u);
 * needs nz >= 2 and 2 (nz - 1) with no prime factor above 7.  inplace: in == out, and the
 * buffer must hold max(real, complex) bytes; real data sits unpadded at the
 * start of the buffer (Sec. 3.1 lists in- and out-of-place transforms).
 *
 * share_only = 1 runs the local stages of the single rank (r1, r2) of the
 * m1 x m2 grid at its Table 1 shapes (Sec. 2, 3.2), the work one GPU of a
 * distributed run does between exchanges.  The user arrays are that rank's
 * blocks alone: forward input its X-pencil, forward output its Z-pencil (and
 * the reverse), in Table 1 order.  Each exchange keeps only the part the rank
 * sends to itself; the blocks the other ranks would send count as zero.  The
 * forward result is thus the 3D transform of the input extended by zeros to
 * the whole grid, restricted to the rank's Z-pencil block; the backward
 * result is the staged C2R of the input extended by zeros, restricted to the
 * rank's X-pencil block.  A 1 x 1 share is the whole transform.  Not
 * combinable with inplace (PF_EUNSUPPORTED).  The workspace holds the
 * global-layout arrays; zero fills stand in for the received blocks.
 *
 * fused_xy = 1 runs the X and Y stages of the transform as one pass, the
 * slab form of the method (Sec. 4.3, Fig. 10: one exchange instead of two
 * while the processor count does not exceed the grid edge, which always holds
 * on one GPU): a persistent kernel transforms each z plane along X and then,
 * once every X tile of the plane is done, along Y, while the plane's X output
 * may still sit in the last-level caches.  A direction then takes two passes
 * (forward: fused X-Y, Z; backward: Z, fused Y-X) and gives the same result
 * up to rounding order (the same arithmetic; tested against the oracle).
 * Built for FP32 plain-math 1 x 1 plans with nx in {1024, 2048} and ny in
 * {512, 1024}; otherwise pf_setup returns PF_EUNSUPPORTED (also if the
 * device's XCDs, which serve one work queue each, cannot be enumerated at
 * setup).  The kernel's waits for other workgroups always end (they wait only
 * for work taken earlier from the same queue) and are also bounded;
 * pf_check_status reports a bound that expired.
 */
typedef struct pf_layout {
    int m1, m2;     /* processor grid, each >= 1                            */
    int stride1;    /* 1 (default) = STRIDE1 defined, 0 = undefined         */
    int useeven;    /* 0 (default) or 1                                     */
    int precision;  /* PF_F32 (default) or PF_F64                           */
    int math;       /* PF_PLAIN (default), PF_MFMA_FP16X2, PF_MFMA_BF16X2   */
    int inplace;    /* 0 (default) = out-of-place, 1 = in-place             */
    int third;      /* PF_THIRD_FFT (default), PF_THIRD_EMPTY, PF_THIRD_CHEB */
    int share_only; /* 0 (default) or 1: one rank's share, see below         */
    int r1, r2;     /* share_only: the rank, 0 <= r1 < m1, 0 <= r2 < m2;     */
                    /* otherwise 0                                            */
    int fused_xy;   /* 0 (default) or 1: X and Y stages in one pass, below   */
} pf_layout;

typedef struct pf_plan pf_plan;

/* Fill *l with the defaults above.  l must not be NULL. */
void pf_layout_init(pf_layout *l);

/*
 * Host-only validation of a grid and layout; touches no GPU.  Checks sizes >= 1,
 * the processor-grid bounds of Eq. 2 read as m1 <= min(nx/2+1, ny) and
 * m2 <= min(ny, nz) (every rank's block in every pencil non-empty), option
 * values, and that every length factors into 2, 3, 5 and 7.
 * Returns PF_OK, PF_EINVAL or PF_EUNSUPPORTED.
 */
int pf_check(int nx, int ny, int nz, const pf_layout *l);

/*
 * Host-only: the block of rank (r1, r2) in the given pencil (Table 1), for a
 * grid and layout that pf_check accepts.  start[3] and size[3] are the global
 * offsets and extents of the block along (X, Y, Z) -- along X in modes for Y-
 * and Z-pencils; order[3] lists the axes (0 = X, 1 = Y, 2 = Z) from fastest to
 * slowest in memory.  An axis of length n split over M ranks gives rank r
 * floor(n/M) + (r < n mod M) elements starting at r floor(n/M) + min(r, n mod M)
 * (blocks differ by at most one, Sec. 3.4).
 */
int pf_query_dims(int nx, int ny, int nz, const pf_layout *l, int pencil, int r1, int r2, int start[3],
                  int size[3], int order[3]);

/*
 * Create a plan: validates (as pf_check), factors the three lengths, builds
 * the twiddle tables in FP64 on the host (rounded once to the plan's
 * precision), uploads them, and allocates the workspace on the current HIP
 * device.  On success *out holds the plan; on failure *out is NULL.
 */
int pf_setup(int nx, int ny, int nz, const pf_layout *l, pf_plan **out);

/* pf_query_dims for the plan's grid and layout. */
int pf_get_dims(const pf_plan *p, int pencil, int r1, int r2, int start[3], int size[3], int order[3]);

/* Bytes of device workspace the plan needs (0 for a NULL plan). */
size_t pf_workspace_bytes(const pf_plan *p);

/*
 * Use caller-owned device memory as the workspace instead of the plan's own
 * (which is freed).  ws must be 256-byte aligned and hold at least
 * pf_workspace_bytes(p) bytes; it must outlive the plan's use.
 */
int pf_set_workspace(pf_plan *p, void *ws, size_t bytes);

/*
 * Forward transform (R2C): real X-pencil `in` -> complex Z-pencil `out`
 * (layouts above).  Out-of-place plans leave `in` unchanged.  Asynchronous on
 * `stream`.
 */
int pf_ftran_r2c(pf_plan *p, const void *in, void *out, void *stream);

/*
 * Backward transform (C2R): complex Z-pencil `in` -> real X-pencil `out`,
 * unnormalised.  Out-of-place plans leave `in` unchanged.  Asynchronous.
 */
int pf_btran_c2r(pf_plan *p, const void *in, void *out, void *stream);

/*
 * For callers that cannot allocate device memory at call time: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * forward (dir = PF_DIR_FORWARD, as pf_ftran_r2c) or backward (PF_DIR_BACKWARD,
 * as pf_btran_c2r) transform with the same arguments, layouts and results, but
 * with a static device array of the library (PF_NOALLOC_MAX_BYTES bytes per
 * device, held from the first plan made on a device until the process ends) as
 * the workspace instead of the plan's.  The call allocates nothing: no device
 * memory, no events (per-pass timing is not recorded for it), no library
 * buffers; it only enqueues the transform's kernels on `stream`.
 *
 * Limits and errors: PF_EWORKSPACE if the plan's workspace
 * (pf_workspace_bytes) exceeds PF_NOALLOC_MAX_BYTES (FP32 1 x 1 plans up to
 * e.g. 480 x 360 x 250 or 256^3 fit); PF_EUNSUPPORTED for share-only plans;
 * otherwise as pf_ftran_r2c / pf_btran_c2r.  Every call on one device shares
 * that device's array, so calls that overlap in time on one device (two
 * streams, two threads) race and give undefined results; the caller
 * serialises them.  The array keeps the last call's contents; no transform
 * depends on its initial contents.
 */
#define PF_NOALLOC_MAX_BYTES ((size_t)256 << 20)
int pf_exec_noalloc(pf_plan *p, int dir, const void *in, void *out, void *stream);

/* Free the plan's device tables and owned workspace.  NULL is accepted. */
int pf_destroy(pf_plan *p);

/* Static description of a status code. */
const char *pf_strerror(int code);

/*
 * Waits for the device to finish all queued work, then returns PF_ETIMEOUT if
 * a fused X-Y pass of the plan had a wait reach its bound since the last call
 * (its output is then wrong), PF_OK otherwise, and clears the report.
 * PF_OK for plans without fused passes; PF_EINVAL for NULL.
 */
int pf_check_status(pf_plan *p);

/* ---- single passes, for stage-level testing ----------------------------- */

/*
 * Number of HBM passes (kernel launches) one transform makes in direction dir
 * (PF_DIR_FORWARD or PF_DIR_BACKWARD): 3 for a 1 x 1 grid, 5 for m1 * m2 > 1
 * (a pack pass before and an unpack pass after the three transform passes).
 * Share-only plans: 5 forward (zero fill, X, Y, Z, copy of the Z block out)
 * and 6 backward (zero fill, copy of the Z block in, Z, Y, zeroing of the
 * modes outside the rank's kx range, X).
 */
int pf_num_passes(const pf_plan *p, int dir);

/*
 * Run pass `pass` of direction `dir` alone.  Between transform passes the
 * data lives in the workspace layout: complex [nz][nkb][ny][B] where B = 128
 * bytes / complex size (16 for F32, 8 for F64), nkb = ceil(nxh / B), and mode
 * kx of line (y, z) sits at [z][kx / B][y][kx % B]; slots with kx >= nxh are
 * unused.  For a 1 x 1 grid -- forward: pass 0 X stage (user real ->
 * workspace), pass 1 Y stage (workspace in place), pass 2 Z stage (workspace ->
 * user complex); backward: pass 0 Z stage (user complex -> workspace), pass 1 Y
 * stage (in place), pass 2 X stage (workspace -> user real).  For m1 * m2 > 1
 * the transform passes are 1 .. 3 and read / write the global arrays
 * ([nz][ny][nx] real, the 1 x 1 Z-pencil layout complex); pass 0 packs the
 * user's blocks into the global array and pass 4 unpacks the global array into
 * the user's blocks.  `in`/`out` that name the workspace may be any buffer of
 * pf_workspace_bytes bytes.  Share-only plans run their passes only as a
 * whole chain (pf_run_pass returns PF_EUNSUPPORTED).  pass_name returns a
 * short static name.
 */
int pf_run_pass(pf_plan *p, int dir, int pass, const void *in, void *out, void *stream);
const char *pf_pass_name(const pf_plan *p, int dir, int pass);

/*
 * Layout of the workspace between the transform passes of direction dir:
 * PF_WS_BLOCKED, the [nz][nkb][ny][B] rows above, or PF_WS_TRANSPOSED,
 * complex [nz][nxh][ny] (mode kx of line (y, z) at [z][kx][y]: rows of 16
 * lines at one mode, 128 bytes FP32, 256 bytes FP64).  Both chains of a plain STRIDE1 1 x 1 plan with
 * a power-of-two X pass (FP32: nx in {512, 1024, 2048}; FP64: nx in {512,
 * 1024}) and ny a multiple of 16 up to 512 use the transposed form: backward,
 * the Z pass reads adjacent Z-pencil lines per tile, the Y pass runs in place
 * along contiguous lines and the X pass reads the rows of one tile's 16
 * lines; forward (FP64: at nx = 512), mirrored (X writes the rows, Y runs
 * along the lines, Z writes adjacent Z-pencil lines): the same two transposes
 * of Sec. 2, placed differently.  Returns PF_EINVAL for a NULL plan or a bad
 * dir.
 */
#define PF_WS_BLOCKED 0
#define PF_WS_TRANSPOSED 1
int pf_workspace_layout(const pf_plan *p, int dir);

/*
 * Kernel family that runs pass `pass` of direction `dir` (a short static
 * string, "" for an invalid plan / dir / pass): "c2c_generic", "r2c_generic",
 * "c2r_generic" (radix plan read at run time, Sec. 2's 1D transforms as a
 * stage loop); "c2c_pow2", "r2c_pow2", "c2r_pow2" (power-of-two lengths, radix
 * plan fixed at compile time, persistent workgroups); "c2c_mixed",
 * "r2c_mixed", "c2r_mixed" (7-smooth lengths with a compile-time two-step
 * plan, FP32); "xy_fused" (fused_xy); "remap", "fill", "box" (reorders of
 * the processor-grid and share-only plans).  Introspection only.
 */
const char *pf_pass_kernel(const pf_plan *p, int dir, int pass);

/*
 * Algorithmic HBM bytes of one pass: every element read once and written once
 * (real side N * s, complex side nx/2+1 modes * ny * nz * 2s).
 */
double pf_pass_bytes(const pf_plan *p, int dir, int pass);

/* ---- HBM roofline probe --------------------------------------------------- */

/*
 * Plain device-to-device copy of `bytes` bytes (a multiple of 16, both
 * pointers 16-byte aligned, non-overlapping), enqueued on `stream`.  It is the
 * measured ceiling for the memory term of the paper's cost model (Eq. 3: the
 * bytes each element moves divided by the memory bandwidth): every transform
 * pass moves its array once in and once out, as this copy does.  Returns
 * PF_EINVAL for NULL pointers, PF_EALIGN for misaligned pointers or sizes.
 */
int pf_copy(void *dst, const void *src, size_t bytes, void *stream);

/*
 * Bandwidth probes for the memory term of Eq. 3, in the access shapes of the
 * transform passes (bytes a multiple of 16, pointers 16-byte aligned):
 *   PF_PROBE_COPY           pf_copy's one-shot copy (dst != src);
 *   PF_PROBE_TILES          persistent workgroups copy 128 KB tiles, the next
 *                           tile's loads in flight while the current one is
 *                           stored, nontemporal accesses (dst != src): the
 *                           shape of a pass between two arrays;
 *   PF_PROBE_TILES_INPLACE  the same with dst == src, each tile read and
 *                           written back: the shape of the in-place Y pass.
 * Returns PF_EINVAL (NULL pointers, unknown kind), PF_EALIGN, PF_EALIAS (dst
 * and src equal or not as the kind requires), PF_EHIP.
 */
#define PF_PROBE_COPY 0
#define PF_PROBE_TILES 1
#define PF_PROBE_TILES_INPLACE 2
int pf_probe(int kind, void *dst, const void *src, size_t bytes, void *stream);

/* ---- per-pass timing with HIP events ------------------------------------ */

/*
 * enable != 0: every later transform call records a HIP event pair around
 * each of its passes on the call's stream.  enable == 0 stops recording.
 * Either way the accumulated totals are cleared.
 */
int pf_set_timing(pf_plan *p, int enable);

/*
 * Waits for the recorded events, then returns the summed elapsed time in
 * milliseconds and the number of recorded launches of pass `pass` of
 * direction `dir` since timing was enabled.
 */
int pf_get_timing(pf_plan *p, int dir, int pass, double *total_ms, long long *count);

/* ---- differentiable spectral step (Chebyshev third transform) ------------ */

/*
 * For a plan with third = PF_THIRD_CHEB (1 x 1, out-of-place): out = L in with
 *   L u = s B( m * F(u) ),  F = pf_ftran_r2c, B = pf_btran_c2r,
 *   m(kx, ky, kz) = i kx' * (-1 / (kx'^2 + ky'^2 + kz'^2)), m(0) = 0,
 *   kx' = 2 pi kx / nx, ky' = 2 pi ky / ny (ky taken in -ny/2 .. ny/2),
 *   kz' = pi kz / (nz - 1) (the DCT index read as a cosine-series wavenumber),
 *   s = 1 / (nx ny 2 (nz - 1)),
 * i.e. the x derivative of the inverse Laplacian in spectral space.  With
 * adjoint = 1, out = L^T in for the real inner product, computed as
 * s W B( conj(m) * F(W^-1 in) ) with W the DCT end-node weights along z
 * (1 at z = 0 and nz - 1, 2 inside): the adjoint of the type-I DCT is
 * W C W^-1, and the interior-mode factors of the R2C / C2R adjoints cancel.
 * in, out: real [nz][ny][nx]; spec: complex Z-pencil buffer of the plan
 * (caller-owned scratch, contents unspecified on return).  All distinct
 * (PF_EALIAS), 16-byte aligned.  PF_EUNSUPPORTED for other plans.
 * FP32 plans whose extension length 2 (nz - 1) is 256 .. 4096 run the z part
 * (forward DCT, product, backward DCT, and the adjoint's weights, which act
 * along z only and commute with the X and Y stages) as one pass on the
 * plan's workspace; the spectrum is then never written to spec.
 */
int pf_spectral_step(pf_plan *p, const void *in, void *spec, void *out, int adjoint, void *stream);

/* ---- batched transforms ------------------------------------------------ */

/*
 * Many independent 3D transforms of different sizes run together (the same
 * method per transform, Sec. 2; the paper's "any grid dimensions", Sec. 3.1).
 * An axis whose length has a compile-time mixed-radix kernel (the 7-smooth
 * lengths 48 .. 320 but 256, and 360, 480; FP32) runs that kernel; every
 * other axis runs the runtime-radix kernels (the power-of-two kernels, whose
 * persistent grids are sized per transform, are not used in a batch).  A
 * fused pass is one kernel launch per group of transforms that share a
 * kernel -- the runtime-radix passes grouped by block size, the mixed-radix
 * passes by length -- over the tiles of every transform of the group (a
 * device table maps each workgroup to its transform).
 *
 * pf_tune: per axis (x, y, z) a radix order (0: radix 16 first, then 8, 4, 2,
 * 3, 5, 7; 1: 8, 4, 2, 3, 5, 7; 2: 4, 2, 3, 5, 7; 3: 3, 5, 7 first, then 16,
 * 8, 4, 2) and a tile width (0: the default, else at most that many line
 * pairs per X tile or columns per Y / Z tile; below 16 it selects the
 * runtime-radix kernel for that axis).  Chosen per transform by the
 * package's autotuner; NULL means defaults.
 */
typedef struct pf_tune {
    int radix_order[3];
    int tile[3];
} pf_tune;

typedef struct pf_batch pf_batch;

#define PF_BATCH_SERIAL 0  /* transform after transform, three launches each   */
#define PF_BATCH_FUSED 1   /* per pass, one launch per block size over all transforms (default) */
#define PF_BATCH_GRAPH 2   /* flag: replay the direction from a captured hipGraph */
#define PF_BATCH_STREAMS 4 /* flag: spread independent launches over the batch's own streams */

/*
 * dims: count triples (nx, ny, nz).  l: precision, stride1 and third as for
 * pf_setup; m1 = m2 = 1, out-of-place, plain math only (else
 * PF_EUNSUPPORTED).  tune: NULL or count entries.  The batch owns its
 * plans, tables and workspace.  Errors as pf_setup, for the first transform
 * that fails.
 */
int pf_batch_setup(int count, const int *dims, const pf_layout *l, const pf_tune *tune, pf_batch **out);

/*
 * The user arrays of a batch are two device buffers: REAL holds every
 * transform's X-pencil [nz][ny][nx] and COMPLEX every transform's Z-pencil
 * (layout as pf_setup's), each at a 256-byte aligned offset.  which = 0:
 * real, 1: complex.  pf_batch_offset returns transform i's byte offset
 * ((size_t)-1 on bad arguments), pf_batch_bytes the buffer's total size.
 */
size_t pf_batch_offset(const pf_batch *b, int which, int i);
size_t pf_batch_bytes(const pf_batch *b, int which);

/*
 * mode: PF_BATCH_SERIAL or PF_BATCH_FUSED, optionally | PF_BATCH_GRAPH: the
 * first call of a direction with given buffers captures its launches into a
 * hipGraph (on a stream of the batch's own) and every call replays it on the
 * caller's stream; new buffers or a new mode are captured again (after the
 * caller's stream has drained the old graph).  PF_BATCH_STREAMS (not with
 * PF_BATCH_GRAPH): the call forks PF_BATCH_NSTREAMS streams of the batch's
 * own from the caller's stream (an event recorded there), runs independent
 * work on them -- whole transforms, largest first, each on the least loaded
 * stream (serial), or the launch groups of one pass (fused; the streams join
 * between passes) -- and joins them back into the caller's stream, so that
 * small launches of different transforms overlap.  Work queued on the
 * caller's stream afterwards sees the results.  Returns PF_EINVAL for values
 * outside 0 .. 7, PF_EUNSUPPORTED for PF_BATCH_GRAPH | PF_BATCH_STREAMS.
 */
#define PF_BATCH_NSTREAMS 4
int pf_batch_set_mode(pf_batch *b, int mode);

/*
 * Forward: in = REAL buffer (read only), out = COMPLEX buffer; backward the
 * reverse.  Both 256-byte aligned (PF_EALIGN), distinct (PF_EALIAS).
 * Asynchronous on `stream`; one batch must not run on two streams at once.
 */
int pf_batch_ftran_r2c(pf_batch *b, const void *in, void *out, void *stream);
int pf_batch_btran_c2r(pf_batch *b, const void *in, void *out, void *stream);
int pf_batch_destroy(pf_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* PENCILFFT_H */
