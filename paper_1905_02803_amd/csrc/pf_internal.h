// pf_internal.h -- declarations shared by the host planner (capi.hip) and the
// transform kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace pf {

constexpr int kMaxStages = 16;  // radix stages of one 1D length
constexpr int kEMax = 16;       // complex elements per thread per stage (F32; F64 uses half)
constexpr int kMaxLds = 128 * 1024;  // dynamic LDS any kernel may request
// threads per block of the generic kernels: the tile chooser keeps TC x wpc
// <= 512, and n <= 8192 (FP32) / 4096 (FP64) keeps wpc <= 512 at TC = 1
constexpr int kGenericThreads = 512;

// Mixed-radix plan of one 1D length n = radix[0] * radix[1] * ...
// Stage s has Ns = radix[0] * ... * radix[s-1] and reads its twiddles
// W_{Ns R}^{r k} (k < Ns, 1 <= r < R) at twoff[s] + k (R - 1) + r - 1.
struct FftSpec {
    int n;
    int nstages;
    int radix[kMaxStages];
    int twoff[kMaxStages];
};

// Address map of one side of a column-tile pass.  Tile (a, cb) holds columns
// cb * TC .. cb * TC + TC - 1 of a grid of C columns; element (c, p) of the
// tile sits at  a*sa + (cb / cpb)*sblk + (cb % cpb)*TC*sc + c*sc + p*sp.
// Blocked workspace sides use cpb = B / TC; linear sides use cpb = CB, sblk = 0.
struct Side {
    long long sa, sblk, sc, sp, cpb;
    int v8;  // power-of-two C2C pass, row side: rows not 16-byte aligned, 8-byte column accesses
};

enum PassKind {
    PASS_C2C = 0,
    PASS_R2C_X = 1,
    PASS_C2R_X = 2,
    PASS_C2C_P2 = 3,
    PASS_R2C_P2 = 4,
    PASS_C2R_P2 = 5,
    PASS_REMAP = 6,
    PASS_FILL = 7,
    PASS_BOX = 8,
    PASS_FUSED_XY = 9,  // launched by the planner from its FusedArgs (p2_fused_launch)
    PASS_C2C_MR = 10,   // compile-time mixed-radix passes (kernels_mr.h), FP32
    PASS_R2C_MR = 11,
    PASS_C2R_MR = 12
};

// Reorder between the global arrays and the concatenated Table 1 pencil
// blocks of an m1 x m2 processor grid (ranks in the order r2 m1 + r1).  Lines
// are whole in every pencil, so the reorder copies lines:
//   REMAP_XPENCIL  real lines (y, z) of length nx;
//   REMAP_ZSTRIDE1 complex lines (kx, ky) of length nz (Z-pencil ZYX);
//   REMAP_ZXYZ     complex row segments (kz, ky, r1) of length b(nxh, m1, r1)
//                  (Z-pencil XYZ).
enum RemapKind { REMAP_XPENCIL = 0, REMAP_ZSTRIDE1 = 1, REMAP_ZXYZ = 2 };

struct RemapArgs {
    const void *src;
    void *dst;
    int kind;
    int gather;  // 1: blocks -> global array, 0: global array -> blocks
    int words;   // 4-byte words per element
    int nx, ny, nz, nxh, m1, m2;
    long long nlines;
};

// Zero elements of the blocked workspace [z][kb][y][B] (rows of 128 bytes):
// rows (z, kb, y) of nbox boxes [z0, z1) x [kb0, kb1) x [y0, y1); within a
// row, the elements whose mode kx = kb B + c lies in [keep0, keep1) are left
// alone.  `words`: 4-byte words per element (2 for FP32 complex, 4 for FP64).
struct FillArgs {
    void *w;
    int words, B, ny;
    long long zrows, kbrows;  // workspace rows between z planes / column blocks
    int keep0, keep1;
    int nbox;
    int z0[4], z1[4], kb0[4], kb1[4], y0[4], y1[4];
};

// Copy a box between a strided global array (dimension 0 contiguous, element
// strides st1, st2 of dimensions 1 and 2) and a dense block [s2][s1][s0]:
// global element (o0 + i0, o1 + i1, o2 + i2) <-> block element (i0, i1, i2).
struct BoxArgs {
    const void *src;
    void *dst;
    int words;
    int to_block;  // 1: global -> block, 0: block -> global
    long long st1, st2;
    int o0, o1, o2, s0, s1, s2;
};

struct PassArgs {
    const void *in;
    void *out;
    const void *tw;  // stage twiddle tables of fft.n, plan precision
    FftSpec fft;
    int tc_log2;   // TC = columns (C2C) or line pairs (X passes) per tile
    int wpc_log2;  // threads per column
    int pitch;     // LDS column pitch in complex elements
    int C;         // valid columns (C2C passes)
    long long A, CB;  // C2C tile grid: A * CB tiles
    Side in_s, out_s;
    int inp, outp;  // power-of-two C2C pass, kind of side: 1 lines, 0 aligned rows, 2 unaligned rows
    int math;       // power-of-two passes: 0 plain, 1 / 2 middle radix-16 stage on MFMA (FP16 / BF16 hi+lo),
                    // 3 (C2C pass) no transform: the reorder alone, 4 (C2C pass) type-I DCT by the
                    // even extension (lines of cheb = fft.n / 2 + 1 points), 5 (fused spectral
                    // step) type-I DCT split once
    int tile_order; // power-of-two C2C pass: 0 tile t = (t / CB, t % CB), 1 tile t = (t % A, t / A)
    int xcd;        // power-of-two C2C pass: 1 to give each XCD runs of consecutive tiles
    int cheb;       // C2C pass: > 0 = lines of cheb points, transformed as their even
                    // extension of length fft.n = 2 (cheb - 1) (type-I DCT); 0 = plain
    // X passes: real lines (y, z) flattened as g = z * ny + y; line g's spectrum
    // is workspace row z zrows + kb kbrows + y0 + y of column block kb
    long long lines;
    long long ld_real;  // elements between consecutive real lines
    int ny, nkb, b_log2, nxh;
    int y0;
    long long zrows, kbrows;
    int xtr;  // backward power-of-two X pass: 1 = transposed rows, mode k of line (y, z) at
              // z zrows + k kbrows + y (rows of 16 lines at one mode; ny a multiple of 16)
};

struct PassDesc {
    PassKind kind;
    RemapArgs r;  // PASS_REMAP only
    FillArgs f;   // PASS_FILL only
    BoxArgs b;    // PASS_BOX only
    int dir;   // -1 forward, +1 backward
    int prec;  // PF_F32 / PF_F64
    unsigned blocks;
    unsigned threads;
    size_t lds;
    PassArgs a;
};

// Work list of one batched pass (generic kernels): transform i owns blocks
// first[i] .. first[i+1] - 1 and runs with args[i] (device tables).  in_user /
// out_user: the pass reads / writes the caller's arrays, and args[i].in /
// .out hold byte offsets from user_in / user_out.
struct BatchArgs {
    const PassArgs *args;
    const long long *first;
    int count;
    int in_user, out_user;
    const char *user_in;
    char *user_out;
};

struct BatchLaunch {
    PassKind kind;
    int dir, prec;
    int n;  // mixed-radix passes: the transform length shared by the launch's transforms
    unsigned blocks, threads;
    size_t lds;
    BatchArgs b;
};

hipError_t launch_batch(const BatchLaunch &L, hipStream_t s);

// Spectral step on a Chebyshev-third Z-pencil half spectrum U (layout of the
// plan): U *= m or conj(m), m = scale * i kx' (-1 / (kx'^2 + ky'^2 + kz'^2)),
// kx' = 2 pi kx / nx, ky' = 2 pi ky / ny (ky signed), kz' = pi kz / (nz - 1);
// m = 0 at k = 0.
struct SpecArgs {
    void *U;
    int nx, ny, nz, nxh, stride1, f64, conj;
    double scale;
};
hipError_t launch_spec_mul(const SpecArgs &a, hipStream_t s);
// dst[z][y][x] = src[z][y][x] * w(z)^e, w = 1 at z = 0 and nz - 1, else 2; e = +1 or -1
hipError_t launch_zweight(const void *src, void *dst, int nx, int ny, int nz, int f64, int e, hipStream_t s);

// Allow every kernel instantiation up to max_lds bytes of dynamic LDS.
hipError_t prepare_kernels(size_t max_lds);
// Enqueue one pass.
hipError_t launch_pass(const PassDesc &d, hipStream_t s);
hipError_t launch_remap(const RemapArgs &r, hipStream_t s);
hipError_t launch_fill(const FillArgs &f, hipStream_t s);
hipError_t launch_box(const BoxArgs &b, hipStream_t s);
// Plain 16-byte-per-lane device copy (bytes a multiple of 16).
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
// Copy in 128 KB tiles by persistent workgroups (src == dst: in place).
hipError_t launch_copy_tiles(const void *src, void *dst, size_t bytes, hipStream_t s);

// Fused X-Y pass (kernels_p2.hip, k_xy_fused): the X and Y stages of every z
// plane in one persistent launch.  x / y: the X and Y passes' arguments (the
// Y side is the blocked workspace, in place).  nq: work queues, one per XCD.
// ctl: nq + nz counters, zeroed before each launch, then a status word (bit
// 0: a wait reached spin_limit).
struct FusedArgs {
    PassArgs x, y;
    unsigned *ctl;
    int nq, lag, nz;
    int xtiles, ytiles;  // 16-line X tiles / Y tiles per plane
    int xitems, yitems;  // work items per plane (an item is 512 threads' worth of tiles)
    long long spin_limit;
};
bool p2_fused_supported(int nx, int ny, int prec);
size_t p2_fused_lds_bytes(int nx, int ny);
int p2_fused_tiles_per_item(int n, int x);  // tiles per item: X (x = 1, n = nx) or Y (x = 0, n = ny)
hipError_t p2_fused_prepare(int nx, int ny);
const void *p2_fused_symbol(int nx, int ny, int fwd);
// Number of XCDs the workgroups of a `blocks`-workgroup launch run on, if they
// are numbered 0 .. n-1 (each a work queue of the fused pass), else 0.
hipError_t p2_xcd_queues(unsigned blocks, int *nq);
hipError_t p2_fused_launch(const FusedArgs &f, int fwd, int nx, int ny, unsigned blocks, hipStream_t s);

// Compile-time mixed-radix passes, FP32 (kernels_mr.hip): the C2C column pass
// (PASS_C2C_MR, 16 columns per tile, a.tc_log2 = 4) and the X passes
// (PASS_R2C_MR / PASS_C2R_MR, mr_x_pairs() line pairs per tile) of a length n the table
// holds; one tile per workgroup.  a.tw: W_n^m, m < n (forward sign).
bool mr_supported(int n, int prec);
int mr_threads_of(int n, int xpass);  // threads per workgroup of the C2C (xpass 0) or X kernel
int mr_x_pairs();                     // line pairs per X tile (a power of two)
size_t mr_lds_bytes(int n, int xpass);
hipError_t mr_launch(const PassDesc &d, hipStream_t s);
hipError_t mr_launch_batch(const BatchLaunch &L, hipStream_t s);

// Power-of-two FP64 C2C pass (kernels_p2.hip, k_c2c_p2d): plain FFT along Y or
// Z, 8 columns per tile, n = 256, 512, 1024; launched by p2_launch.
bool p2d_supported(int n);
size_t p2d_lds_bytes(int n);
int p2d_threads(int n);
hipError_t p2d_prepare(int n);

// Power-of-two FP32 C2C pass (kernels_p2.hip).
bool p2_supported(int n, int prec);
bool p2_has_mfma(int n);  // a matrix-core variant of the length-n pass exists
int p2_tc(int n);
int p2_threads(int n);
size_t p2_lds_bytes(int n, int math);
hipError_t p2_prepare(int n);
int p2_blocks_per_cu(const PassDesc &d);
hipError_t p2_launch(const PassDesc &d, hipStream_t s);
// fused spectral step along z on the workspace (Chebyshev third transform,
// extension length d.a.fft.n = 256 .. 4096, FP32): forward type-I DCT, product
// with the multiplier (its conjugate and the end-node weights when adj), inverse
hipError_t p2_spec_prepare(int n);
int p2_spec_blocks_per_cu(int n, unsigned threads, size_t lds);
hipError_t p2_spec_launch(const PassDesc &d, int adj, int nx, float scale, hipStream_t s);
// the same step with the type-I DCT split once (d.a.math = 5; nz = 257): one
// tile per workgroup, twiddles [L-point table][M-point table][W_4M^k]
bool p2_spec_sr_supported(int nz);
unsigned p2_spec_sr_threads(int nz);
size_t p2_spec_sr_lds_bytes(int nz);
// Even power-of-two X stage (fft.n of the pass is nx / 2): FP32 for nx = 512 ..
// 2048 (tiles of 16 lines), FP64 for nx = 512, 1024 (tiles of 8 lines, 16 on
// the transposed workspace).
// (tr: the pass reads / writes the transposed workspace; FP64 tiles are then 16 lines)
bool p2x_supported(int nx, int prec);
int p2x_threads(int nx, int prec, int tr);
int p2x_tile_lines(int prec, int tr);
size_t p2x_lds_bytes(int nx, int math, int prec, int tr);
hipError_t p2x_prepare(int nx, int prec);

// LDS index with one pad slot every 16 complex elements (spreads the strided
// Stockham writes over the banks).
__host__ __device__ inline int pidx(int i) { return i + (i >> 4); }

}  // namespace pf
