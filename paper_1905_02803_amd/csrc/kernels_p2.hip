// kernels_p2.hip -- C2C column-tile pass for power-of-two lengths, FP32.
//
// Same job as k_c2c_tile (one Y or Z stage of the transpose-based 3D FFT,
// Sec. 2, with the pencil re-orientation folded into the address maps), but
// with the radix plan fixed at compile time (N = 16 * 16 * R, or 16 * R for
// N <= 256) so that:
//   * the first radix-16 stage reads its 16 inputs straight from HBM into
//     registers (the elements q, q + N/16, ... of a column are exactly the
//     inputs of butterfly q) and the last stage writes straight from
//     registers to HBM -- LDS is used only for the exchanges in between;
//   * every thread holds 16 points of one column in every stage, so each
//     stage reads and writes the same point set {q + (N/16) m};
//   * the block is persistent: while it transforms tile t it already has
//     the loads of its next tile in flight (register double buffering);
//   * a tile is 16 columns of a 16-wide workspace block (128-byte rows).
// Thread roles: on a side whose columns are contiguous (rows of the tile are
// contiguous) lanes run along columns; on a side whose points are contiguous
// (whole lines) lanes run along points.  Middle stages always run along
// columns.  The LDS tile uses a swizzle that keeps every one of these access
// patterns free of bank conflicts for N = 1024.
#include <type_traits>
#include <vector>

#include "fft_device.h"
#include "fused_schedule.h"
#include "pf_internal.h"

namespace pf {

// ---- streaming global accesses ----------------------------------------------
// Each pass reads and writes every element once.  Access sites may carry the
// nontemporal hint (no reuse expected in the caches); which sites do is fixed
// at compile time by the bits of PF_STREAM_MASK.  The default streams every
// store except the row stores of a pass with a point-major input side, and
// the row loads of the Y / Z passes: on MI355X at 1024^3 the Y passes gain
// about 25%, the X passes about 5%; streaming the remaining sites was slower.
#ifndef PF_STREAM_MASK
#define PF_STREAM_MASK 0x3Du
#endif
enum : unsigned {
    ST_C2C_ROWS = 1,       // Y / Z pass: 16-byte stores of rows, row-major input side
    ST_C2C_ROWS_INP = 2,   // Y / Z pass: 16-byte stores of rows, point-major input side
    ST_C2C_POINTS = 4,     // Y / Z pass: 8-byte stores to a point-major output side
    ST_R2C = 8,            // forward X pass: stores to the workspace
    ST_C2R = 16,           // backward X pass: stores of real lines
    LD_C2C_ROWS = 32,      // Y / Z pass: 16-byte loads of rows
    LD_R2C = 64,           // forward X pass: loads of real lines
    LD_C2R = 128,          // backward X pass: loads from the workspace
    LD_C2C_POINTS = 256,   // Y / Z pass: 8-byte loads from a point-major input side
    ST_C2C_UROWS = 512,    // Z pass: 8-byte stores to rows that are not 16-byte aligned
};
template <unsigned BIT>
constexpr bool streamed() {
    return (PF_STREAM_MASK & BIT) != 0;
}

// XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round-robin
// (block b on XCD b % 8); with it on, each full round of G = gridDim.x tiles
// is permuted so that XCD x works on the G / 8 consecutive tiles x G/8 ..
// (x+1) G/8 - 1.  Neighbouring tiles then share one L2, which merges the
// partial cache lines they both write when rows are not line aligned.  The
// last, partial round keeps the identity order.
__device__ __forceinline__ int xcd_tile(int t, int ntiles, int on) {
    const int G = (int)gridDim.x;
    if (!on || (G & 7)) return t;
    const int k = t / G, b = t - k * G;
    if ((k + 1) * G > ntiles) return t;
    return k * G + (b & 7) * (G >> 3) + (b >> 3);
}

// threadIdx.x passed through an empty asm statement: lane indices and LDS
// addresses derived from it are then recomputed inside a tile loop instead of
// being hoisted and held (or spilled) across it
__device__ __forceinline__ int opaque_tid() {
    int v = threadIdx.x;
    asm volatile("" : "+v"(v));
    return v;
}

typedef float pf_f4 __attribute__((ext_vector_type(4)));
typedef float pf_f2 __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ void gst(float4 *p, float4 v) {
    if constexpr (NT) {
        const pf_f4 u = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(u, reinterpret_cast<pf_f4 *>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ void gst(float2 *p, float2 v) {
    if constexpr (NT) {
        const pf_f2 u = {v.x, v.y};
        __builtin_nontemporal_store(u, reinterpret_cast<pf_f2 *>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ float4 gld(const float4 *p) {
    if constexpr (NT) {
        const pf_f4 u = __builtin_nontemporal_load(reinterpret_cast<const pf_f4 *>(p));
        return make_float4(u.x, u.y, u.z, u.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ float2 gld(const float2 *p) {
    if constexpr (NT) {
        const pf_f2 u = __builtin_nontemporal_load(reinterpret_cast<const pf_f2 *>(p));
        return make_float2(u.x, u.y);
    } else {
        return *p;
    }
}

typedef double pf_d2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void gst_d(double2 *p, double2 v) {
    if constexpr (NT) {
        const pf_d2 u = {v.x, v.y};
        __builtin_nontemporal_store(u, reinterpret_cast<pf_d2 *>(p));
    } else {
        *p = v;
    }
}
template <bool NT>
__device__ __forceinline__ double2 gld_d(const double2 *p) {
    if constexpr (NT) {
        const pf_d2 u = __builtin_nontemporal_load(reinterpret_cast<const pf_d2 *>(p));
        return make_double2(u.x, u.y);
    } else {
        return *p;
    }
}

extern __shared__ __align__(16) unsigned char pf_smem[];

__host__ __device__ constexpr int p2_stages(int N) { return N <= 256 ? 2 : 3; }
__host__ __device__ constexpr int p2_radix(int N, int s) {
    return s == 0 ? 16 : (N <= 256 ? N / 16 : (s == 1 ? 16 : N / 256));
}
__host__ __device__ constexpr int p2_ns(int N, int s) { return s == 0 ? 1 : (s == 1 ? 16 : 256); }
// offset of stage s in the twiddle table (entries Ns (R - 1) per stage)
__host__ __device__ constexpr int p2_twoff(int N, int s) {
    return s == 0 ? 0 : p2_twoff(N, s - 1) + p2_ns(N, s - 1) * (p2_radix(N, s - 1) - 1);
}

// LDS slot (in 16-byte column pairs) of point p, pair cp; TC/2 pairs per row.
// Bank behaviour of gfx950 as the SQ_LDS_BANK_CONFLICT counter shows it:
// 16-byte reads serve 16 lanes per cycle from 64 banks of 4 bytes, 16-byte
// writes 8 lanes per cycle from 32 banks (8-byte accesses: twice the lanes).
// The row xor (bit 0 of the row from bits 3, 7, 8 of p) and the pair xor
// (bits 0-2 of p ^ p >> 4 ^ p >> 5) make every exchange of the Y / Z kernels
// and of the matrix-core stage conflict-free under that model for N = 256 ..
// 1024 and 16 columns; only the mirrored (k, M - k) accesses of the X
// stages' split keep some two-way conflicts.
template <int TC>
__device__ __forceinline__ int p2_slot(int p, int cp) {
    constexpr int CP = TC / 2;
    const int row = p ^ (((p >> 3) ^ (p >> 7) ^ (p >> 8)) & 1);
    return row * CP + (cp ^ ((p ^ (p >> 4) ^ (p >> 5)) & (CP - 1)));
}

// One stage's butterflies on the 16 registers of each of a thread's two
// columns: butterfly i (j = q + i N/16) takes v[i + r 16/R], r < R, twiddles
// by W_{NS R}^{r k}, k = j mod NS, and leaves its R outputs in the same
// registers.  Each twiddle is read once and applied to both columns.
template <int N, int R, int NS, int DIR>
__device__ __forceinline__ void p2_butterflies2(cx<float> (&v0)[16], cx<float> (&v1)[16], int q,
                                                const cx<float> *tws) {
    constexpr int T = N / 16;
    constexpr int BPT = 16 / R;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = q + i * T;
        const int k = j & (NS - 1);
        cx<float> w0[R], w1[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w0[r] = v0[i + r * BPT];
            w1[r] = v1[i + r * BPT];
        }
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<float> t = tws[k * (R - 1) + r - 1];
                if (DIR > 0) t.y = -t.y;
                w0[r] = cmul(w0[r], t);
                w1[r] = cmul(w1[r], t);
            }
        }
        Dft<float, R, DIR>::run(w0);
        Dft<float, R, DIR>::run(w1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v0[i + r * BPT] = w0[r];
            v1[i + r * BPT] = w1[r];
        }
    }
}

__device__ __forceinline__ float4 pack2(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }

// ---- radix-16 stage as DFT-matrix products on the matrix cores ------------
// For 16 butterflies at once (the MFMA's 16 columns) the radix-16 DFT
// Y[k] = sum_r W16^{DIR r k} X[r] is the real product C = A B with K = 32
// interleaving real and imaginary parts (K index 2r + c):
//   B[2r + c][b] = (Re, Im)[c] of X_b[r],
//   Ar[k][2r] = cos,  Ar[k][2r+1] = -DIR sin   (C = Re Y)
//   Ai[k][2r] = DIR sin, Ai[k][2r+1] = cos     (C = Im Y),  angle 2 pi r k / 16.
// v_mfma_f32_16x16x32 lane l holds A[l%16][8(l/16) .. +8), B[8(l/16) .. +8)[l%16]
// and returns C[4(l/16) .. +4)[l%16]: lane (b, g) brings points 4g .. 4g+3 of
// butterfly b and receives outputs 4g .. 4g+3 of it.  Both operands are split
// into a high and a low half-precision part; hi*hi + hi*lo + lo*hi is
// accumulated in FP32.  With FP16's 11-bit significands the dropped lo*lo term
// and the residual of the two-term split are about 2^-22 of the product, below
// FP32 rounding; with BF16's 8 bits both are about 2^-16, which sets the BF16
// form's error floor (about 5e-6 relative L2 over a 3D transform).  FP16 inputs
// are first scaled by a power of two per butterfly (largest component in
// [1, 2)); BF16 keeps FP32's exponent range and needs no scale.
typedef _Float16 mf_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 mf_b8 __attribute__((ext_vector_type(8)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
constexpr size_t kMfmaTableBytes = 64 * 4 * 16;  // A operands: 4 vectors of 16 bytes per lane

// cos(2 pi m / 16) for any integer m (closed forms cos(pi/8), cos(pi/4),
// sin(pi/8)), by selects: no runtime-indexed table in private memory.
__device__ __forceinline__ float cos16(int m) {
    const int a = m & 15;
    const int f = a <= 8 ? a : 16 - a;  // cos is even: fold to 0 .. 8
    const float c1 = (float)kCosPi8, c2 = (float)kSqrtHalf, c3 = (float)kSinPi8;
    const float mag = f == 0 || f == 8 ? 1.f : f == 1 || f == 7 ? c1 : f == 2 || f == 6 ? c2 : f == 3 || f == 5 ? c3 : 0.f;
    return f > 4 ? -mag : mag;
}
__device__ __forceinline__ float sin16(int m) { return cos16(m - 4); }

template <int MT>
struct MfmaSplit;
template <>
struct MfmaSplit<1> {  // FP16 hi + lo
    typedef mf_h8 vec;
    typedef _Float16 elem;
    __device__ static void split(float x, _Float16 &h, _Float16 &l) {
        h = (_Float16)x;
        l = (_Float16)(x - (float)h);
    }
    __device__ static mf_f4 mma(vec a, vec b, mf_f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct MfmaSplit<2> {  // BF16 hi + lo
    typedef mf_b8 vec;
    typedef __bf16 elem;
    __device__ static void split(float x, __bf16 &h, __bf16 &l) {
        h = (__bf16)x;
        l = (__bf16)(x - (float)h);
    }
    __device__ static mf_f4 mma(vec a, vec b, mf_f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

// The constant A operands of a lane (row k = l % 16, K = 8 (l/16) + e).  They
// are built once per block into LDS (4 vectors per lane, 4 KB) and read back
// only inside the matrix-core stage.
template <int DIR, int MT>
struct MfmaDft16 {
    typedef typename MfmaSplit<MT>::vec vec;
    vec arh, arl, aih, ail;
    __device__ void init(int lane) {
        const int k = lane & 15, g = lane >> 4;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int r = 4 * g + (e >> 1);
            const float c = cos16(r * k), sn = (float)DIR * sin16(r * k);
            const float ar = (e & 1) ? -sn : c;
            const float ai = (e & 1) ? c : sn;
            typename MfmaSplit<MT>::elem h, l;
            MfmaSplit<MT>::split(ar, h, l);
            arh[e] = h;
            arl[e] = l;
            MfmaSplit<MT>::split(ai, h, l);
            aih[e] = h;
            ail[e] = l;
        }
    }
    __device__ void store(vec *t, int lane) const {
        t[4 * lane] = arh;
        t[4 * lane + 1] = arl;
        t[4 * lane + 2] = aih;
        t[4 * lane + 3] = ail;
    }
    __device__ void load(const vec *t, int lane) {
        arh = t[4 * lane];
        arl = t[4 * lane + 1];
        aih = t[4 * lane + 2];
        ail = t[4 * lane + 3];
    }
    // x: this lane's 4 inputs (points 4g .. 4g+3) of butterfly l % 16; returns the outputs 4g .. 4g+3.
    __device__ void run(cx<float> (&x)[4]) const {
        float sc = 1.f;
        int ex = 127;
        if (MT == 1) {  // per-butterfly power-of-two scale: largest |component| into [1, 2)
            float m = 0.f;
#pragma unroll
            for (int s = 0; s < 4; ++s) m = fmaxf(m, fmaxf(fabsf(x[s].x), fabsf(x[s].y)));
            m = fmaxf(m, __shfl_xor(m, 16));
            m = fmaxf(m, __shfl_xor(m, 32));
            ex = m > 0.f ? ((__float_as_int(m) >> 23) & 255) : 127;
            ex = min(max(ex, 1), 253);
            sc = __int_as_float((254 - ex) << 23);  // 2^(127 - ex), exact
        }
        vec bh, bl;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            typename MfmaSplit<MT>::elem h, l;
            MfmaSplit<MT>::split(x[s].x * sc, h, l);
            bh[2 * s] = h;
            bl[2 * s] = l;
            MfmaSplit<MT>::split(x[s].y * sc, h, l);
            bh[2 * s + 1] = h;
            bl[2 * s + 1] = l;
        }
        mf_f4 cr = {0.f, 0.f, 0.f, 0.f}, ci = {0.f, 0.f, 0.f, 0.f};
        cr = MfmaSplit<MT>::mma(arh, bh, cr);
        ci = MfmaSplit<MT>::mma(aih, bh, ci);
        cr = MfmaSplit<MT>::mma(arh, bl, cr);
        ci = MfmaSplit<MT>::mma(aih, bl, ci);
        cr = MfmaSplit<MT>::mma(arl, bh, cr);
        ci = MfmaSplit<MT>::mma(ail, bh, ci);
        const float inv = MT == 1 ? __int_as_float(ex << 23) : 1.f;  // 2^(ex - 127)
#pragma unroll
        for (int s = 0; s < 4; ++s) x[s] = make_float2(cr[s] * inv, ci[s] * inv);
    }
};

// Stage 1 (radix 16, NS = 16) of an N-point column FFT on the LDS tile, on the
// matrix cores.  Wave w takes butterflies q = 8w .. 8w+7 of all 16 columns;
// within a group lane (b, g) holds column b, points q + (N/16)(4g + s).
// Twiddles W_{256}^{r (q mod 16)} are applied in FP32 before the product.
// Butterfly q reads and writes only LDS rows congruent to q mod 8, so the
// groups 0-3 and 4-7 of all waves touch disjoint rows: each half is read,
// synchronised, transformed and written in turn (half the live operands).
template <int N, int TC, int DIR, int MT>
__device__ __forceinline__ void p2_stage1_mfma(float4 *buf, const cx<float> *tws,
                                               const typename MfmaSplit<MT>::vec *atab, int tid) {
    constexpr int T = N / 16;
    static_assert(TC == 16, "the matrix-core stage takes 16 columns");
    const int lane = tid & 63, w = tid >> 6;
    MfmaDft16<DIR, MT> dft;
    dft.load(atab, lane);
    const int b = lane & 15, g = lane >> 4;
    float2 *lds2 = reinterpret_cast<float2 *>(buf);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        cx<float> x[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 8 * w + 4 * h + i;
#pragma unroll
            for (int s = 0; s < 4; ++s) x[i][s] = lds2[2 * p2_slot<TC>(q + T * (4 * g + s), b >> 1) + (b & 1)];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 8 * w + 4 * h + i;
            const int k = q & 15;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int r = 4 * g + s;
                if (r > 0 && k > 0) {
                    cx<float> t = tws[k * 15 + r - 1];
                    if (DIR > 0) t.y = -t.y;
                    x[i][s] = cmul(x[i][s], t);
                }
            }
            dft.run(x[i]);
            const int base = (q - k) * 16 + k;
#pragma unroll
            for (int s = 0; s < 4; ++s) lds2[2 * p2_slot<TC>(base + 16 * (4 * g + s), b >> 1) + (b & 1)] = x[i][s];
        }
    }
    __syncthreads();
}

// Stage 0 (radix 16, no twiddles) of an N-point column FFT on the matrix
// cores, fed from registers.  Each wave runs 8 groups of 16 butterflies; in
// group i, lane (b, g) holds points q + (N/16)(4g + s), s < 4, of butterfly
// (column, q) in x[4 i + s] -- for a side whose columns are contiguous (LINES =
// false) the group's butterflies are the 16 columns at q = 8w + i, for a side
// whose points are contiguous (LINES = true) they are 16 consecutive q of one
// column (group j = 8w + i: column j / (N/256), q = 16 (j mod N/256) + b), so
// that either way 16 lanes read one 128-byte run.  The outputs r = 4g + s land
// on points 16 q + r of the LDS tile.
template <int N, bool LINES>
__device__ __forceinline__ void p2_mfma_group(int w, int i, int b, int &col, int &q) {
    if constexpr (LINES) {
        const int j = 8 * w + i;
        col = j / (N / 256);
        q = 16 * (j % (N / 256)) + b;
    } else {
        col = b;
        q = 8 * w + i;
    }
}

template <int N, int TC, int DIR, int MT, bool LINES>
__device__ __forceinline__ void p2_stage0_mfma(cx<float> (&x)[32], float4 *buf,
                                               const typename MfmaSplit<MT>::vec *atab, int tid) {
    static_assert(TC == 16, "the matrix-core stage takes 16 columns");
    const int lane = tid & 63, w = tid >> 6;
    const int b = lane & 15, g = lane >> 4;
    MfmaDft16<DIR, MT> dft;
    dft.load(atab, lane);
    float2 *lds2 = reinterpret_cast<float2 *>(buf);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        cx<float> y[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) y[s] = x[4 * i + s];
        dft.run(y);
        int col, q;
        p2_mfma_group<N, LINES>(w, i, b, col, q);
#pragma unroll
        for (int s = 0; s < 4; ++s) lds2[2 * p2_slot<TC>(16 * q + 4 * g + s, col >> 1) + (col & 1)] = y[s];
    }
}

// Stage 0 on the matrix cores with its inputs in the LDS tile (the backward X
// stage, whose inputs come from the inverse split): every group's inputs are
// read before any output is written (outputs of butterfly q cover all rows
// 16 q .. 16 q + 15, so rows of different waves' butterflies interleave).
template <int N, int TC, int DIR, int MT>
__device__ __forceinline__ void p2_stage0_mfma_lds(float4 *buf, const typename MfmaSplit<MT>::vec *atab, int tid) {
    constexpr int T = N / 16;
    const int lane = tid & 63, w = tid >> 6;
    const int b = lane & 15, g = lane >> 4;
    const float2 *lds2 = reinterpret_cast<const float2 *>(buf);
    cx<float> x[32];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int q = 8 * w + i;
#pragma unroll
        for (int s = 0; s < 4; ++s) x[4 * i + s] = lds2[2 * p2_slot<TC>(q + T * (4 * g + s), b >> 1) + (b & 1)];
    }
    __syncthreads();
    p2_stage0_mfma<N, TC, DIR, MT, false>(x, buf, atab, tid);
    __syncthreads();
}

// Trade values between the lanes of points q (even) and q + 1 (odd), which are
// cp_lanes apart in the wave, so that the row-major layout (v0, v1) = (column
// 2 cp, column 2 cp + 1) of the lane's own point and the column-major layout
// (v0, v1) = (row q & ~1, row q | 1) of the lane's own column are exchanged;
// the map is its own inverse.  Even lane: keeps v0, swaps v1; odd lane: keeps
// v1, swaps v0.
__device__ __forceinline__ void pair_swap(cx<float> (&v0)[16], cx<float> (&v1)[16], bool odd, int cp_lanes) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const float2 a0 = v0[m], a1 = v1[m];
        const float2 give = make_float2(odd ? a0.x : a1.x, odd ? a0.y : a1.y);
        const float2 got = make_float2(__shfl_xor(give.x, cp_lanes), __shfl_xor(give.y, cp_lanes));
        v0[m] = make_float2(odd ? got.x : a0.x, odd ? got.y : a0.y);
        v1[m] = make_float2(odd ? a1.x : got.x, odd ? a1.y : got.y);
    }
}

// Each thread owns a pair of adjacent columns (2 cp, 2 cp + 1) and 16 points
// q + (N/16) m of both.  INP / OUTP, the kind of that side: 1 if its points
// are contiguous (lines), 0 if its columns are (rows, 16-byte column-pair
// accesses), 2 for rows that are not 16-byte aligned (8-byte accesses).
template <int N, int TC, int DIR, int INP, int OUTP, int MT>
__global__ __launch_bounds__(N / 16 * TC / 2) void k_c2c_p2(PassArgs a) {
    constexpr int T = N / 16;
    constexpr int CP = TC / 2;
    constexpr int NT = T * CP;
    constexpr int S = p2_stages(N);
    constexpr int RL = p2_radix(N, S - 1);
    constexpr int NSL = p2_ns(N, S - 1);
    float4 *buf = reinterpret_cast<float4 *>(pf_smem);
    cx<float> *twl = reinterpret_cast<cx<float> *>(buf + N * CP);
    const int tid = threadIdx.x;
    const cx<float> *__restrict__ tw = reinterpret_cast<const cx<float> *>(a.tw);
    for (int i = tid; i < N - 1; i += NT) twl[i] = tw[i];
    constexpr bool MC = MT == 1 || MT == 2;  // middle stage on the matrix cores
    // stage 0 on the matrix cores too, fed from the load registers, where the
    // input side is aligned rows (INP 0) or lines (INP 1)
    constexpr bool MC0 = MC && (INP == 0 || INP == 1);
    typedef typename MfmaSplit<MC ? MT : 1>::vec avec;
    avec *atab = reinterpret_cast<avec *>(twl + N);  // matrix-core A operands (MC)
    if constexpr (MC) {
        if (tid < 64) {
            MfmaDft16<DIR, MT> d0;
            d0.init(tid);
            d0.store(atab, tid);
        }
    }

    const cx<float> *__restrict__ in = reinterpret_cast<const cx<float> *>(a.in);
    cx<float> *__restrict__ out = reinterpret_cast<cx<float> *>(a.out);
    const int CB = (int)a.CB;
    const int ntiles = (int)(a.A * a.CB);
    const long long in_step = a.in_s.sp * T;
    const long long out_step = a.out_s.sp * T;
    // MT == 4, the type-I DCT of the a.cheb = N / 2 + 1 points of a side line
    // (Sec. 3.1) as the N-point DFT of its even extension: point j of the
    // extension is stored point j or N - j, and only points j < a.cheb are written
    constexpr bool CH = MT == 4;
    const int nsrc = CH ? a.cheb : N;
    // offset of extension point j from the address of point q (q = j mod T)
    auto ext = [&](int j, int q, long long sp) -> long long {
        return (long long)((CH && j >= nsrc ? N - j : j) - q) * sp;
    };

    // element (column 2 cp, point q) of tile t on a side, and the valid column count
    const int A = (int)a.A;
    auto side_addr = [&](const Side &sd, int t, int cp, int q, int &ncol) -> long long {
        // tile order 1 walks the outer index fastest: concurrently resident
        // tiles then touch different lines of a side whose lines are far apart
        const int ta = a.tile_order ? t % A : t / CB;
        const int cb = a.tile_order ? t / A : t - ta * CB;
        ncol = min(TC, a.C - cb * TC);
        return (long long)ta * sd.sa + (long long)(cb / sd.cpb) * sd.sblk + (long long)(cb % sd.cpb) * TC * sd.sc +
               (long long)(2 * cp) * sd.sc + (long long)q * sd.sp;
    };
    auto load = [&](cx<float>(&d0)[16], cx<float>(&d1)[16], int t) {
        const int tv = opaque_tid();
        if constexpr (MC0) {
            // matrix-core stage 0: group i of the wave in d0[4 i + s] (i < 4) or
            // d1[4 (i - 4) + s], lane (b, g) point q + T (4 g + s) of its column
            const int lane = tv & 63, w = tv >> 6, bl = lane & 15, g = lane >> 4;
            int ncol;
            const long long base = side_addr(a.in_s, t, 0, 0, ncol);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int col, q;
                p2_mfma_group<N, INP == 1>(w, i, bl, col, q);
                if (col < ncol) {
                    const long long e = base + (long long)col * a.in_s.sc + (long long)q * a.in_s.sp;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const cx<float> *src = in + e + (long long)(4 * g + s) * in_step;
                        const float2 v = INP == 1 ? gld<streamed<LD_C2C_POINTS>()>(src)
                                                  : gld<streamed<LD_C2C_ROWS>()>(src);
                        if (i < 4) d0[4 * i + s] = v;
                        else d1[4 * (i - 4) + s] = v;
                    }
                }
            }
            return;
        }
        const int cp_in = INP == 1 ? tv / T : tv % CP;
        const int q_in = INP == 1 ? tv % T : tv / CP;
        int ncol;
        const long long b = side_addr(a.in_s, t, cp_in, q_in, ncol);
        if constexpr (INP == 1) {  // two lines, 8 bytes per lane each
            if (2 * cp_in < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    d0[m] = gld<streamed<LD_C2C_POINTS>()>(in + b + (CH ? ext(q_in + T * m, q_in, 1) : m * in_step));
            }
            if (2 * cp_in + 1 < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    d1[m] = gld<streamed<LD_C2C_POINTS>()>(in + b + a.in_s.sc +
                                                           (CH ? ext(q_in + T * m, q_in, 1) : m * in_step));
            }
        } else if constexpr (INP == 2) {
            // rows not 16-byte aligned: 8-byte column accesses, each instruction
            // covering 16 adjacent columns of one row -- the lane of point q even
            // takes column 2 cp of rows q and q + 1, its partner (q odd, CP lanes
            // away) column 2 cp + 1 of the same rows; swapped into place in the
            // tile loop (pair_swap)
            const bool odd = q_in & 1;
            const int col = 2 * cp_in + (odd ? 1 : 0);
            if (col < ncol) {
                const long long e = b + (odd ? a.in_s.sc - a.in_s.sp : 0);  // column col, row q & ~1
                const int q0 = q_in & ~1;
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    if constexpr (CH) {
                        d0[m] = gld<streamed<LD_C2C_ROWS>()>(in + e + ext(q0 + T * m, q0, a.in_s.sp));
                        d1[m] = gld<streamed<LD_C2C_ROWS>()>(in + e + ext(q0 + 1 + T * m, q0, a.in_s.sp));
                    } else {
                        d0[m] = gld<streamed<LD_C2C_ROWS>()>(in + e + m * in_step);
                        d1[m] = gld<streamed<LD_C2C_ROWS>()>(in + e + a.in_s.sp + m * in_step);
                    }
                }
            }
        } else if (2 * cp_in < ncol) {  // rows: both columns in one 16-byte load
            // a partially valid pair only occurs on a side padded to whole 16-column blocks
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const long long o = CH ? ext(q_in + T * m, q_in, a.in_s.sp) : m * in_step;
                const float4 x = gld<streamed<LD_C2C_ROWS>()>(reinterpret_cast<const float4 *>(in + b + o));
                d0[m] = make_float2(x.x, x.y);
                d1[m] = make_float2(x.z, x.w);
            }
        }
    };

    int t = blockIdx.x;
    cx<float> p0[16], p1[16];
    if constexpr (MC0) {  // lanes of columns past the grid's edge compute on zeros
#pragma unroll
        for (int m = 0; m < 16; ++m) p0[m] = p1[m] = make_float2(0.f, 0.f);
    }
    if (t < ntiles) load(p0, p1, xcd_tile(t, ntiles, a.xcd));
    __syncthreads();  // twiddle table in LDS
    for (; t < ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        const int cp_in = INP == 1 ? tv / T : tv % CP;
        const int q_in = INP == 1 ? tv % T : tv / CP;
        const int cp_mid = tv % CP;
        const int q_mid = tv / CP;
        const int cp_out = OUTP == 1 ? tv / T : tv % CP;
        const int q_out = OUTP == 1 ? tv % T : tv / CP;
        cx<float> v0[16], v1[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            v0[m] = p0[m];
            v1[m] = p1[m];
        }
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(p0, p1, xcd_tile(tn, ntiles, a.xcd));
        if constexpr (INP == 2) pair_swap(v0, v1, q_in & 1, CP);

        if constexpr (MT == 3) {  // no transform (the empty third transform): points keep their index
#pragma unroll
            for (int m = 0; m < 16; ++m) buf[p2_slot<TC>(q_in + T * m, cp_in)] = pack2(v0[m], v1[m]);
            __syncthreads();
        } else if constexpr (MC0) {  // stage 0 on the matrix cores, from the load registers
            cx<float> x[32];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                x[m] = v0[m];
                x[16 + m] = v1[m];
            }
            p2_stage0_mfma<N, TC, DIR, MT, INP == 1>(x, buf, atab, tv);
            __syncthreads();
        } else {
            // stage 0: radix 16 on x[q + T r], outputs to points 16 q + r
            Dft<float, 16, DIR>::run(v0);
            Dft<float, 16, DIR>::run(v1);
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q_in * 16 + r, cp_in)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }

        if constexpr (MT == 3) {
        } else if constexpr (S == 3 && MC) {  // stage 1 on the matrix cores
            p2_stage1_mfma<N, TC, DIR, MT>(buf, twl + p2_twoff(N, 1), atab, tv);
        } else if constexpr (S == 3) {  // stage 1: radix 16, NS = 16
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            p2_butterflies2<N, 16, 16, DIR>(v0, v1, q_mid, twl + p2_twoff(N, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(base + r * 16, cp_mid)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }

        // last stage: outputs land on points q + T m of the thread's columns
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float4 x = buf[p2_slot<TC>(q_out + T * m, cp_out)];
            v0[m] = make_float2(x.x, x.y);
            v1[m] = make_float2(x.z, x.w);
        }
        if constexpr (MT != 3) p2_butterflies2<N, RL, NSL, DIR>(v0, v1, q_out, twl + p2_twoff(N, S - 1));
        {
            int ncol;
            const long long b = side_addr(a.out_s, xcd_tile(t, ntiles, a.xcd), cp_out, q_out, ncol);
            if constexpr (OUTP == 1) {
                if (2 * cp_out < ncol) {
#pragma unroll
                    for (int m = 0; m < 16; ++m)
                        if (!CH || q_out + T * m < nsrc) gst<streamed<ST_C2C_POINTS>()>(out + b + m * out_step, v0[m]);
                }
                if (2 * cp_out + 1 < ncol) {
#pragma unroll
                    for (int m = 0; m < 16; ++m)
                        if (!CH || q_out + T * m < nsrc)
                            gst<streamed<ST_C2C_POINTS>()>(out + b + a.out_s.sc + m * out_step, v1[m]);
                }
            } else if constexpr (OUTP == 2) {  // rows not 16-byte aligned: as the loads, in reverse
                const bool odd = q_out & 1;
                pair_swap(v0, v1, odd, CP);
                const int col = 2 * cp_out + (odd ? 1 : 0);
                if (col < ncol) {
                    const long long e = b + (odd ? a.out_s.sc - a.out_s.sp : 0);
                    const int q0 = q_out & ~1;
#pragma unroll
                    for (int m = 0; m < 16; ++m) {
                        if (!CH || q0 + T * m < nsrc) gst<streamed<ST_C2C_UROWS>()>(out + e + m * out_step, v0[m]);
                        if (!CH || q0 + 1 + T * m < nsrc)
                            gst<streamed<ST_C2C_UROWS>()>(out + e + a.out_s.sp + m * out_step, v1[m]);
                    }
                }
            } else if (2 * cp_out < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    if (!CH || q_out + T * m < nsrc)
                        gst<streamed<INP == 1 ? ST_C2C_ROWS_INP : ST_C2C_ROWS>()>(
                            reinterpret_cast<float4 *>(out + b + m * out_step), pack2(v0[m], v1[m]));
            }
        }
        __syncthreads();  // the next tile's stage 0 overwrites the LDS tile
    }
}

// ---- FP64: the same column-tile pass with one column per thread ------------
// A 128-byte workspace row holds 8 complex doubles, so an FP64 tile is 8
// columns; each thread owns one column (16-byte accesses) and the 16 points
// q + (N/16) m of it in every stage, as the FP32 kernel owns a column pair.
// The LDS slot map is the FP32 kernel's with the column in place of the pair
// (16-byte slots, 8 per row).  Rows (INP / OUTP 0) and lines (1); FP64 rows
// are always 16-byte aligned.
template <int N, int R, int NS, int DIR>
__device__ __forceinline__ void p2_butterflies1(cx<double> (&v)[16], int q, const cx<double> *tws) {
    constexpr int T = N / 16;
    constexpr int BPT = 16 / R;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = q + i * T;
        const int k = j & (NS - 1);
        cx<double> w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = v[i + r * BPT];
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<double> t = tws[k * (R - 1) + r - 1];
                if (DIR > 0) t.y = -t.y;
                w[r] = cmul(w[r], t);
            }
        }
        Dft<double, R, DIR>::run(w);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i + r * BPT] = w[r];
    }
}

template <int N, int DIR, int INP, int OUTP>
__global__ __launch_bounds__(N / 16 * 8) void k_c2c_p2d(PassArgs a) {
    constexpr int TC = 8;
    constexpr int T = N / 16;
    constexpr int NT = T * TC;
    constexpr int S = p2_stages(N);
    constexpr int RL = p2_radix(N, S - 1);
    constexpr int NSL = p2_ns(N, S - 1);
    typedef cx<double> cd;
    cd *buf = reinterpret_cast<cd *>(pf_smem);  // N x 8 slots of 16 bytes
    cd *twl = buf + N * TC;
    const int tid = threadIdx.x;
    const cd *__restrict__ tw = reinterpret_cast<const cd *>(a.tw);
    for (int i = tid; i < N - 1; i += NT) twl[i] = tw[i];
    const cd *__restrict__ in = reinterpret_cast<const cd *>(a.in);
    cd *__restrict__ out = reinterpret_cast<cd *>(a.out);
    const int CB = (int)a.CB, A = (int)a.A;
    const int ntiles = (int)(a.A * a.CB);
    const long long in_step = a.in_s.sp * T;
    const long long out_step = a.out_s.sp * T;
    // slot of (point p, column c): the FP32 map with 8 slots per row
    auto slot = [](int p, int c) { return p2_slot<16>(p, c); };
    // element (column c, point q) of tile t on a side, and the valid column count
    auto side_addr = [&](const Side &sd, int t, int c, int q, int &ncol) -> long long {
        const int ta = a.tile_order ? t % A : t / CB;
        const int cb = a.tile_order ? t / A : t - ta * CB;
        ncol = min(TC, a.C - cb * TC);
        return (long long)ta * sd.sa + (long long)(cb / sd.cpb) * sd.sblk + (long long)(cb % sd.cpb) * TC * sd.sc +
               (long long)c * sd.sc + (long long)q * sd.sp;
    };
    auto load = [&](cd(&d)[16], int t) {
        const int tv = opaque_tid();
        const int c = INP == 1 ? tv / T : tv % TC;
        const int q = INP == 1 ? tv % T : tv / TC;
        int ncol;
        const long long b = side_addr(a.in_s, t, c, q, ncol);
        if (c < ncol) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const double2 *src = reinterpret_cast<const double2 *>(in + b + m * in_step);
                d[m] = INP == 1 ? *src : gld_d<streamed<LD_C2C_ROWS>()>(src);
            }
        }
    };

    int t = blockIdx.x;
    cd p[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) p[m] = make_double2(0.0, 0.0);
    if (t < ntiles) load(p, xcd_tile(t, ntiles, a.xcd));
    __syncthreads();  // twiddle table in LDS
    for (; t < ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        const int c_in = INP == 1 ? tv / T : tv % TC;
        const int q_in = INP == 1 ? tv % T : tv / TC;
        const int c_mid = tv % TC, q_mid = tv / TC;
        const int c_out = OUTP == 1 ? tv / T : tv % TC;
        const int q_out = OUTP == 1 ? tv % T : tv / TC;
        cd v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = p[m];
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(p, xcd_tile(tn, ntiles, a.xcd));
        // stage 0: radix 16 on x[q + T r], outputs to points 16 q + r
        Dft<double, 16, DIR>::run(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[slot(q_in * 16 + r, c_in)] = v[r];
        __syncthreads();
        if constexpr (S == 3) {  // stage 1: radix 16, NS = 16
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_mid + T * m, c_mid)];
            __syncthreads();
            p2_butterflies1<N, 16, 16, DIR>(v, q_mid, twl + p2_twoff(N, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[slot(base + r * 16, c_mid)] = v[r];
            __syncthreads();
        }
        // last stage: outputs land on points q + T m of the thread's column
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_out + T * m, c_out)];
        p2_butterflies1<N, RL, NSL, DIR>(v, q_out, twl + p2_twoff(N, S - 1));
        {
            int ncol;
            const long long b = side_addr(a.out_s, xcd_tile(t, ntiles, a.xcd), c_out, q_out, ncol);
            if (c_out < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    double2 *dst = reinterpret_cast<double2 *>(out + b + m * out_step);
                    if constexpr (OUTP == 1) gst_d<streamed<ST_C2C_POINTS>()>(dst, v[m]);
                    else gst_d<streamed<INP == 1 ? ST_C2C_ROWS_INP : ST_C2C_ROWS>()>(dst, v[m]);
                }
            }
        }
        __syncthreads();  // the next tile's stage 0 overwrites the LDS tile
    }
}

// ---- fused spectral step along z (Chebyshev third transform, Sec. 3.1) -----
// All stages of one N-point column FFT on a tile whose rows are 16-byte column
// pairs on both sides (thread point set q + T m, pair cp, in every stage):
// inputs x[q + T m] in (v0, v1), outputs X[q + T m] in the same registers.
// Ends after the last stage's LDS reads; the caller synchronises before the
// LDS tile is written again.
template <int N, int TC, int DIR>
__device__ __forceinline__ void p2_rows_fft(cx<float> (&v0)[16], cx<float> (&v1)[16], float4 *buf,
                                            const cx<float> *twl, int q, int cp) {
    constexpr int T = N / 16;
    constexpr int S = p2_stages(N);
    constexpr int RL = p2_radix(N, S - 1);
    constexpr int NSL = p2_ns(N, S - 1);
    Dft<float, 16, DIR>::run(v0);
    Dft<float, 16, DIR>::run(v1);
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q * 16 + r, cp)] = pack2(v0[r], v1[r]);
    __syncthreads();
    if constexpr (S == 3) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float4 x = buf[p2_slot<TC>(q + T * m, cp)];
            v0[m] = make_float2(x.x, x.y);
            v1[m] = make_float2(x.z, x.w);
        }
        __syncthreads();
        p2_butterflies2<N, 16, 16, DIR>(v0, v1, q, twl + p2_twoff(N, 1));
        const int k = q & 15;
        const int base = (q - k) * 16 + k;
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(base + r * 16, cp)] = pack2(v0[r], v1[r]);
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const float4 x = buf[p2_slot<TC>(q + T * m, cp)];
        v0[m] = make_float2(x.x, x.y);
        v1[m] = make_float2(x.z, x.w);
    }
    p2_butterflies2<N, RL, NSL, DIR>(v0, v1, q, twl + p2_twoff(N, S - 1));
}

// The spectral step's z part on the blocked workspace after the forward X and
// Y stages, in place, one tile (ky line, 16 kx columns) at a time: the type-I
// DCT of the nz = N / 2 + 1 rows (the N-point DFT of their even extension),
// the product with m = i mu, mu = -scale kx' / (kx'^2 + ky'^2 + kz'^2)
// (conj(m) when ADJ), mu = 0 at k = 0, and the inverse DFT of the product --
// still an even sequence, so its first nz points are the backward type-I DCT.
// kx' = 2 pi kx / nx, ky' = 2 pi ky / ny (ky signed), kz' = 2 pi kz / N with
// kz = min(k, N - k).  The adjoint's end-node weights w(z) (1 at z = 0 and
// nz - 1, 2 inside) act along z only and so commute with the X and Y stages:
// rows are divided by w(z) on load and multiplied by w(z) on store.  The
// spectrum never leaves the block.  a.A = ny lines, a.CB column tiles, a.C =
// nxh valid columns, a.in_s the workspace side, a.cheb = nz; a.out the workspace.
template <int N, int TC, int ADJ>
__global__ __launch_bounds__(N / 16 * TC / 2) void k_spec_p2(PassArgs a, int nx, float scale) {
    constexpr int T = N / 16;
    constexpr int CP = TC / 2;
    constexpr int NT = T * CP;
    float4 *buf = reinterpret_cast<float4 *>(pf_smem);
    cx<float> *twl = reinterpret_cast<cx<float> *>(buf + N * CP);
    const int tid = threadIdx.x;
    const cx<float> *__restrict__ tw = reinterpret_cast<const cx<float> *>(a.tw);
    for (int i = tid; i < N - 1; i += NT) twl[i] = tw[i];
    cx<float> *__restrict__ ws = reinterpret_cast<cx<float> *>(a.out);
    const int nz = a.cheb;
    const int CB = (int)a.CB;
    const int ny = (int)a.A;
    const int ntiles = (int)(a.A * a.CB);
    const Side &sd = a.in_s;
    // workspace address of (tile t, pair cp, row 0) and the tile's valid column count
    auto tile_base = [&](int t, int cp, int &ncol) -> long long {
        const int ta = t / CB, cb = t - ta * CB;
        ncol = min(TC, a.C - cb * TC);
        return (long long)ta * sd.sa + (long long)(cb / sd.cpb) * sd.sblk + (long long)(cb % sd.cpb) * TC * sd.sc +
               (long long)(2 * cp) * sd.sc;
    };
    auto load = [&](cx<float>(&d0)[16], cx<float>(&d1)[16], int t) {
        const int tv = opaque_tid();
        const int cp = tv % CP, q = tv / CP;
        int ncol;
        const long long b = tile_base(t, cp, ncol);
        if (2 * cp < ncol) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = q + T * m;
                const int z = j < nz ? j : N - j;  // the even extension
                const float4 x = gld<streamed<LD_C2C_ROWS>()>(reinterpret_cast<const float4 *>(ws + b + z * sd.sp));
                d0[m] = make_float2(x.x, x.y);
                d1[m] = make_float2(x.z, x.w);
            }
        }
    };

    int t = blockIdx.x;
    cx<float> p0[16], p1[16];
    if (t < ntiles) load(p0, p1, t);
    __syncthreads();  // twiddle table in LDS
    const float two_pi = 6.283185307179586f;
    const float kyf = two_pi / (float)ny, kxf = two_pi / (float)nx, kzf = two_pi / (float)N;
    const float sg = ADJ ? -1.f : 1.f;
    for (; t < ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        const int cp = tv % CP, q = tv / CP;
        cx<float> v0[16], v1[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            v0[m] = p0[m];
            v1[m] = p1[m];
        }
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(p0, p1, tn);
        if constexpr (ADJ) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int j = q + T * m;
                const int z = j < nz ? j : N - j;
                const float w = (z == 0 || z == nz - 1) ? 1.f : 0.5f;
                v0[m] = make_float2(v0[m].x * w, v0[m].y * w);
                v1[m] = make_float2(v1[m].x * w, v1[m].y * w);
            }
        }
        p2_rows_fft<N, TC, -1>(v0, v1, buf, twl, q, cp);
        {
            const int ta = t / CB, cb = t - ta * CB;
            const int kx0 = cb * TC + 2 * cp;
            const int kys = 2 * ta <= ny ? ta : ta - ny;
            const float kyr = kyf * (float)kys;
            const float kx0r = kxf * (float)kx0, kx1r = kxf * (float)(kx0 + 1);
            const float r0 = kx0r * kx0r + kyr * kyr, r1 = kx1r * kx1r + kyr * kyr;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int k = q + T * m;
                const float kzr = kzf * (float)(2 * k <= N ? k : N - k);
                const float kz2 = kzr * kzr;
                // 1 / |k|^2 by the hardware reciprocal (1 ulp): the step's FP32
                // error budget is set by the transforms, not by this product
                const float k20 = r0 + kz2, k21 = r1 + kz2;
                const float mu0 = k20 > 0.f ? sg * (-scale * kx0r) * __builtin_amdgcn_rcpf(k20) : 0.f;
                const float mu1 = sg * (-scale * kx1r) * __builtin_amdgcn_rcpf(k21);  // kx0 + 1 > 0
                v0[m] = make_float2(-mu0 * v0[m].y, mu0 * v0[m].x);
                v1[m] = make_float2(-mu1 * v1[m].y, mu1 * v1[m].x);
            }
        }
        __syncthreads();  // the inverse transform rewrites the LDS tile
        p2_rows_fft<N, TC, 1>(v0, v1, buf, twl, q, cp);
        {
            int ncol;
            const long long b = tile_base(t, cp, ncol);
            if (2 * cp < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int j = q + T * m;
                    if (j < nz) {
                        float4 x = pack2(v0[m], v1[m]);
                        if constexpr (ADJ) {
                            const float w = (j == 0 || j == nz - 1) ? 1.f : 2.f;
                            x = make_float4(x.x * w, x.y * w, x.z * w, x.w * w);
                        }
                        gst<streamed<ST_C2C_ROWS>()>(reinterpret_cast<float4 *>(ws + b + j * sd.sp), x);
                    }
                }
            }
        }
        __syncthreads();  // the next tile's stage 0 overwrites the LDS tile
    }
}

// The same z part with the type-I DCT split once (split radix), for nz = 257
// (L = nz - 1 = 256, M = L / 2).  For a column x_0 .. x_L:
//  * the even outputs Y_{2m}, m = 0 .. M, are the L-point DFT of the even
//    sequence a_n = x_n + x_{L-n}, n < L (a_0 = x_0 + x_L);
//  * the odd outputs Y_{2m+1}, m < M, are the type-III DCT
//    B_m = sum_{k<M} X_k cos(pi k (2m+1) / (2M)) of X_0 = c_0, X_k = 2 c_k,
//    c_k = x_k - x_{L-k}; it is one M-point DFT, v = DFT_M(V) of V_0 = c_0,
//    V_k = W_{4M}^k (c_k + i c_{M-k}), read out as B_{2j} = v_j and
//    B_{2j+1} = v_{M-1-j} (the transpose of the DFT-based type-II DCT, which
//    holds for complex data because each step is complex-linear).
// That is 1.5 L points of DFT per column where the even extension takes 2 L,
// with no running sum (the half-length form with one carries FP32 rounding
// across the column).  The L-point DFTs run on the first L/16 x 8 threads
// (group L), the M-point ones on the next M/16 x 8 (group M), side by side,
// with the barriers at the top level; each transform stages the tile's L + 1
// rows in LDS once, and the two DFT exchanges then reuse that space.  One
// tile (ky line, 16 kx columns) per workgroup.  The multiplier, the adjoint's
// weights and the arguments are those of k_spec_p2 (with a.xtr set, the tile
// is 16 adjacent ky at one kx of the transposed workspace); a.tw holds the L-point
// stage table, the M-point stage table (each padded to L and M entries) and
// W_{4M}^k, k < M.
template <int L, int ADJ>
__global__ __launch_bounds__(L / 16 * 8 + L / 32 * 8) void k_spec_sr(PassArgs a, int nx, float scale) {
    static_assert(L == 256, "two-stage DFTs of L and L / 2 points");
    constexpr int TC = 16, CP = TC / 2;
    constexpr int M = L / 2;
    constexpr int TL = L / 16, TM = M / 16;
    constexpr int NL = TL * CP, NT = NL + TM * CP;
    constexpr int NLOAD = ((L + 1) * CP + NT - 1) / NT;  // staging loads per thread
    static_assert(NL % 64 == 0 && NT % CP == 0, "groups are whole waves; a thread's column pair is fixed");
    float4 *stg = reinterpret_cast<float4 *>(pf_smem);  // rows 0 .. L of the tile, [row][pair]
    float4 *bufL = stg;                                 // the DFT exchanges reuse the staging area
    float4 *bufM = stg + L * CP;
    cx<float> *twL = reinterpret_cast<cx<float> *>(stg + (L + M) * CP);
    const cx<float> *twM = twL + L;
    const cx<float> *w4 = twL + L + M;
    const int tid = threadIdx.x;
    const cx<float> *__restrict__ tw = reinterpret_cast<const cx<float> *>(a.tw);
    for (int i = tid; i < L + 2 * M; i += NT) twL[i] = tw[i];
    cx<float> *__restrict__ ws = reinterpret_cast<cx<float> *>(a.out);
    // a.xtr: the tile is 16 adjacent ky at one kx (rows of the transposed
    // workspace: A = nxh lines of kx, C = ny) instead of 16 kx at one ky
    const bool tr = a.xtr != 0;
    const int ny = tr ? a.C : (int)a.A;
    const int CB = (int)a.CB;
    const int t = blockIdx.x;
    const int ta = t / CB, cb = t - ta * CB;
    const int ncol = min(TC, a.C - cb * TC);
    const Side &sd = a.in_s;
    // workspace address of the tile's column pair p, row 0
    auto colbase = [&](int p) -> long long {
        return (long long)ta * sd.sa + (long long)(cb / sd.cpb) * sd.sblk + (long long)(cb % sd.cpb) * TC * sd.sc +
               (long long)(2 * p) * sd.sc;
    };
    {  // stage rows 0 .. L (element f: row f / 8, pair f % 8 = tid % 8)
        const int lp = tid % CP;
        const long long b = colbase(lp);
        const bool live = 2 * lp < ncol;
        float4 xr[NLOAD];
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const int row = tid / CP + i * (NT / CP);
            xr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (live && row <= L)
                xr[i] = gld<streamed<LD_C2C_ROWS>()>(reinterpret_cast<const float4 *>(ws + b + (long long)row * sd.sp));
        }
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const int row = tid / CP + i * (NT / CP);
            if (row <= L) stg[row * CP + lp] = xr[i];
        }
    }
    __syncthreads();

    const bool gl = tid < NL;  // wave-uniform
    const int tg = gl ? tid : tid - NL;
    const int cp = tg % CP, q = tg / CP;
    cx<float> v0[16], v1[16];
    auto sub = [](float4 u, float4 v) { return make_float4(u.x - v.x, u.y - v.y, u.z - v.z, u.w - v.w); };
    // staged row r as the transform reads it: the adjoint's first transform divides
    // rows by w(z) (1 at z = 0 and L, 2 inside); applied here rather than when the
    // rows are staged, which lets the compiler issue every staging load before the
    // first wait
    auto rd = [&](int r, auto first) {
        float4 x = stg[r * CP + cp];
        if constexpr (ADJ && decltype(first)::value) {
            const float w = (r == 0 || r == L) ? 1.f : 0.5f;
            x = make_float4(x.x * w, x.y * w, x.z * w, x.w * w);
        }
        return x;
    };
    // the type-I DCT of the staged rows; group L ends with Y_{2k} at k = q + TL m in
    // (v0[m], v1[m]), group M with v_j at j = q + TM m
    auto dct = [&](auto first) {
        if (gl) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int n = q + TL * m;
                const float4 u = rd(n, first), w = rd(L - n, first);  // n = 0 pairs with row L
                v0[m] = make_float2(u.x + w.x, u.y + w.y);
                v1[m] = make_float2(u.z + w.z, u.w + w.w);
            }
        } else {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const int k = q + TM * m;
                const float4 ck = sub(rd(k, first), rd(L - k, first));
                if (k == 0) {
                    v0[m] = make_float2(ck.x, ck.y);
                    v1[m] = make_float2(ck.z, ck.w);
                } else {
                    const float4 cm = sub(rd(M - k, first), rd(M + k, first));
                    const cx<float> w = w4[k];
                    v0[m] = cmul(w, make_float2(ck.x - cm.y, ck.y + cm.x));
                    v1[m] = cmul(w, make_float2(ck.z - cm.w, ck.w + cm.z));
                }
            }
        }
        __syncthreads();  // the DFT exchanges overwrite the staged rows
        Dft<float, 16, -1>::run(v0);
        Dft<float, 16, -1>::run(v1);
        float4 *buf = gl ? bufL : bufM;
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q * 16 + r, cp)] = pack2(v0[r], v1[r]);
        __syncthreads();
        if (gl) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = bufL[p2_slot<TC>(q + TL * m, cp)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            p2_butterflies2<L, L / 16, 16, -1>(v0, v1, q, twL + p2_twoff(L, 1));
        } else {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = bufM[p2_slot<TC>(q + TM * m, cp)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            p2_butterflies2<M, M / 16, 16, -1>(v0, v1, q, twM + p2_twoff(M, 1));
        }
    };
    // output row of register m: group L holds Y_{2k} (k = q + TL m, kept for k <= M),
    // group M holds B_{2j} = Y_{4j+1} (j < M/2) or B_{2(M-1-j)+1} = Y_{2L-4j-1}
    auto out_row = [&](int m) {
        if (gl) {
            const int k = q + TL * m;
            return k <= M ? 2 * k : -1;
        }
        const int j = q + TM * m;
        return j < M / 2 ? 4 * j + 1 : 2 * L - 4 * j - 1;
    };

    dct(std::true_type());
    {  // product with m = i mu (conj(m) when ADJ), mu = 0 at k = 0
        const float two_pi = 6.283185307179586f;
        const float kyf = two_pi / (float)ny, kxf = two_pi / (float)nx, kzf = two_pi / (float)(2 * L);
        const float sg = ADJ ? -1.f : 1.f;
        auto sky = [ny](int k) { return 2 * k <= ny ? k : k - ny; };  // ky in -ny/2 .. ny/2
        const int c0 = cb * TC + 2 * cp;  // the pair's first column
        // (kx', ky') of the pair's two columns
        const float kx0r = kxf * (float)(tr ? ta : c0), kx1r = kxf * (float)(tr ? ta : c0 + 1);
        const float ky0r = kyf * (float)sky(tr ? c0 : ta), ky1r = kyf * (float)sky(tr ? c0 + 1 : ta);
        const float r0 = kx0r * kx0r + ky0r * ky0r, r1 = kx1r * kx1r + ky1r * ky1r;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int k = out_row(m);
            const float kzr = kzf * (float)(k < 0 ? 0 : k);
            const float kz2 = kzr * kzr;
            // 1 / |k|^2 by the hardware reciprocal (1 ulp), as in k_spec_p2
            const float k20 = r0 + kz2, k21 = r1 + kz2;
            const float mu0 = k20 > 0.f ? sg * (-scale * kx0r) * __builtin_amdgcn_rcpf(k20) : 0.f;
            const float mu1 = k21 > 0.f ? sg * (-scale * kx1r) * __builtin_amdgcn_rcpf(k21) : 0.f;
            v0[m] = make_float2(-mu0 * v0[m].y, mu0 * v0[m].x);
            v1[m] = make_float2(-mu1 * v1[m].y, mu1 * v1[m].x);
        }
    }
    __syncthreads();  // every wave has read the DFT exchanges before the rows are staged again
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int row = out_row(m);
        if (row >= 0) stg[row * CP + cp] = pack2(v0[m], v1[m]);
    }
    __syncthreads();
    // the product is an even sequence again: its first nz points are the backward type-I DCT
    dct(std::false_type());
    if (2 * cp < ncol) {
        const long long b = colbase(cp);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int row = out_row(m);
            if (row >= 0) {
                float4 x = pack2(v0[m], v1[m]);
                if constexpr (ADJ) {
                    const float w = (row == 0 || row == L) ? 1.f : 2.f;
                    x = make_float4(x.x * w, x.y * w, x.z * w, x.w * w);
                }
                gst<streamed<ST_C2C_ROWS>()>(reinterpret_cast<float4 *>(ws + b + (long long)row * sd.sp), x);
            }
        }
    }
}

// ---- X stage for even power-of-two nx, FP32 --------------------------------
// A real line x of length nx = 2M is transformed as the complex line
// z[m] = x[2m] + i x[2m+1] of length M (8-byte loads, half the butterflies),
// then split: with Z = DFT_M(z), E[k] = (Z[k] + conj Z[M-k]) / 2,
// O[k] = (Z[k] - conj Z[M-k]) / (2i), the modes are X[k] = E[k] + W_nx^k O[k]
// for k = 0 .. M (the (nx+2)/2 modes of Sec. 3.2).  The backward transform
// inverts the split, Zb[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k])
// W_nx^-k, after replacing X[0] and X[M] by their real parts (the staged
// complex-to-real transform), and an unnormalised inverse DFT_M returns
// x[2m] + i x[2m+1].  A tile is 16 consecutive lines (8 line pairs); the
// spectra go to / come from the blocked workspace (rows of 16 modes).  Twiddles:
// a.tw holds the M-point stage table (M - 1 entries) and at offset M the
// split table W_nx^k, k = 0 .. M.

// Row offsets in the workspace of the 16 lines of tile t (line g = z ny + y
// starts at row z zrows + y0 + y, column block 0).
__device__ __forceinline__ long long x_rowoff(const PassArgs &a, int g) {
    const int z = g / a.ny;
    const int y = g - z * a.ny;
    return ((long long)z * a.zrows + a.y0 + y) << 4;
}

// The forward X stage split like C2cP2: tables, loads of one tile, transform,
// split and stores of one tile.  tv: the thread's index among the NT threads
// of one tile; buf, rowoff: that tile's LDS work area; tables: twiddles (the
// M-point stage table, then the split table at M), A operands at 2 M + 2.
template <int M, int MT, bool TR = false>
struct R2cP2 {
    static constexpr int TC = 16;
    static constexpr int T = M / 16;
    static constexpr int CP = 8;
    static constexpr int NT = T * CP;
    static constexpr int S = p2_stages(M);
    static constexpr int RL = p2_radix(M, S - 1);
    static constexpr int NSL = p2_ns(M, S - 1);
    static constexpr int NKB = M / 16 + 1;  // workspace column blocks for M + 1 modes
    static constexpr size_t kTileLds = (size_t)M * CP * 16;
    static constexpr size_t kTableLds = (size_t)(2 * M + 2) * 8 + (MT ? kMfmaTableBytes : 0);
    typedef typename MfmaSplit<MT == 0 ? 1 : MT>::vec avec;

    const PassArgs &a;
    float4 *buf;
    cx<float> *twl, *spl;
    avec *atab;  // matrix-core A operands (MT != 0)
    long long *rowoff;
    const float *__restrict__ in;
    cx<float> *__restrict__ out;
    int lines, ntiles;
    long long kbstride;

    __device__ __forceinline__ R2cP2(const PassArgs &pa, float4 *tile_lds, cx<float> *tables, long long *rows) : a(pa) {
        buf = tile_lds;
        twl = tables;
        spl = twl + M;
        atab = reinterpret_cast<avec *>(twl + 2 * M + 2);
        rowoff = rows;
        in = reinterpret_cast<const float *>(a.in);
        out = reinterpret_cast<cx<float> *>(a.out);
        lines = (int)a.lines;
        ntiles = (lines + 15) / 16;
        kbstride = a.kbrows << 4;
    }

    // tables into LDS by nthr threads; the caller synchronises before use
    __device__ __forceinline__ void init_tables(int tv, int nthr) const {
        const cx<float> *__restrict__ tw = reinterpret_cast<const cx<float> *>(a.tw);
        for (int i = tv; i < 2 * M + 1; i += nthr)
            if (i != M - 1) twl[i] = tw[i];
        if constexpr (MT != 0) {
            if (tv < 64) {
                MfmaDft16<-1, MT> d0;
                d0.init(tv);
                d0.store(atab, tv);
            }
        }
    }

    __device__ __forceinline__ void load(cx<float> (&d0)[16], cx<float> (&d1)[16], int t, int tv) const {
        if constexpr (MT != 0) {
            // matrix-core stage 0: group i in d0[4 i + s] (i < 4) or d1[4 (i - 4) + s];
            // lane (b, g) holds complex point q + T (4 g + s) of its line
            const int lane = tv & 63, w = tv >> 6, bl = lane & 15, g = lane >> 4;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                int l, q;
                p2_mfma_group<M, true>(w, i, bl, l, q);
                if (16 * t + l < lines) {
                    const float *pl = in + (long long)(16 * t + l) * a.ld_real + 2 * q;
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float2 v =
                            gld<streamed<LD_R2C>()>(reinterpret_cast<const float2 *>(pl + 2 * T * (4 * g + s)));
                        if (i < 4) d0[4 * i + s] = v;
                        else d1[4 * (i - 4) + s] = v;
                    }
                }
            }
            return;
        }
        const int cp_in = tv / T, q_in = tv % T;  // lines: lanes along points
        const int ga = 16 * t + 2 * cp_in;
        const float *pa = in + (long long)ga * a.ld_real + 2 * q_in;
        if (ga < lines) {
#pragma unroll
            for (int m = 0; m < 16; ++m) d0[m] = gld<streamed<LD_R2C>()>(reinterpret_cast<const float2 *>(pa + 2 * T * m));
        }
        if (ga + 1 < lines) {
#pragma unroll
            for (int m = 0; m < 16; ++m)
                d1[m] = gld<streamed<LD_R2C>()>(reinterpret_cast<const float2 *>(pa + a.ld_real + 2 * T * m));
        }
    }

    // Transform, split and stores of tile t; ends with a barrier (the LDS tile
    // and row offsets are reused by the next tile).
    template <bool NTS = streamed<ST_R2C>()>
    __device__ __forceinline__ void tile(cx<float> (&v0)[16], cx<float> (&v1)[16], int t, int tv) const {
        const int cp_in = tv / T, q_in = tv % T;     // lines: lanes along points
        const int cp_mid = tv % CP, q_mid = tv / CP; // exchanges: lanes along line pairs
        if (tv < 16 && 16 * t + tv < lines) rowoff[tv] = x_rowoff(a, 16 * t + tv);

        if constexpr (MT != 0) {  // stage 0 on the matrix cores, from the load registers
            cx<float> x[32];
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                x[m] = v0[m];
                x[16 + m] = v1[m];
            }
            p2_stage0_mfma<M, TC, -1, MT, true>(x, buf, atab, tv);
        } else {
            Dft<float, 16, -1>::run(v0);
            Dft<float, 16, -1>::run(v1);
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q_in * 16 + r, cp_in)] = pack2(v0[r], v1[r]);
        }
        __syncthreads();
        if constexpr (S == 3 && MT != 0) {
            p2_stage1_mfma<M, TC, -1, MT>(buf, twl + p2_twoff(M, 1), atab, tv);
        } else if constexpr (S == 3) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            p2_butterflies2<M, 16, 16, -1>(v0, v1, q_mid, twl + p2_twoff(M, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(base + r * 16, cp_mid)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
            v0[m] = make_float2(x.x, x.y);
            v1[m] = make_float2(x.z, x.w);
        }
        __syncthreads();
        p2_butterflies2<M, RL, NSL, -1>(v0, v1, q_mid, twl + p2_twoff(M, S - 1));
#pragma unroll
        for (int m = 0; m < 16; ++m) buf[p2_slot<TC>(q_mid + T * m, cp_mid)] = pack2(v0[m], v1[m]);
        __syncthreads();

        // split and store: chunk = (column block kb, line pair pr, mode pair kp)
        // over the first M modes; the chunks of k = 0 also store mode M (alone
        // in the last column block, and computed from Z[0] as mode 0 is)
        auto split = [&](int k, int pr, float2 &xa, float2 &xb) {
            const int kz = k < M ? k : k - M;       // Z is M-periodic
            const int km = k == 0 ? 0 : M - k;      // (M - k) mod M for k <= M
            const float4 zk = buf[p2_slot<TC>(kz < M ? kz : 0, pr)];
            const float4 zm = buf[p2_slot<TC>(km < M ? km : 0, pr)];
            const cx<float> w = spl[k <= M ? k : M];
            // line a: (zk.x, zk.y), (zm.x, zm.y); line b: .z, .w
            const float2 Ea = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            const float2 Oa = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
            const float2 Eb = make_float2(0.5f * (zk.z + zm.z), 0.5f * (zk.w - zm.w));
            const float2 Ob = make_float2(0.5f * (zk.w + zm.w), 0.5f * (zm.z - zk.z));
            xa = cadd(Ea, cmul(w, Oa));
            xb = cadd(Eb, cmul(w, Ob));
        };
        if constexpr (TR) {
            // transposed rows: mode k of line g = z ny + y at z zrows + k kbrows + y
            // (zrows = nxh ny, kbrows = ny, ny a multiple of 16), so one row holds the
            // tile's 16 lines at one mode.  Item f: line pair pr = f & 7 (lanes along
            // the row), mode k = f >> 3 < M; the items of k = 0 also store mode M.
            const int g0 = 16 * t;
            const int z0 = g0 / a.ny;
            const int y0 = g0 - z0 * a.ny;
            cx<float> *tb = out + (long long)z0 * a.zrows + y0;
            const int ks = (int)a.kbrows;
            for (int f = tv; f < M * 8; f += NT) {
                const int pr = f & 7, k = f >> 3;
                float2 xa, xb;
                split(k, pr, xa, xb);
                gst<NTS>(reinterpret_cast<float4 *>(tb + (k * ks + 2 * pr)), pack2(xa, xb));
                if (k == 0) {
                    split(M, pr, xa, xb);
                    gst<NTS>(reinterpret_cast<float4 *>(tb + (M * ks + 2 * pr)), pack2(xa, xb));
                }
            }
            __syncthreads();  // the LDS tile is reused by the next tile
            return;
        }
        for (int f = tv; f < (NKB - 1) * 64; f += NT) {
            const int kb = f >> 6, pr = (f >> 3) & 7, kp = f & 7;
            const int ga = 16 * t + 2 * pr;
            const int k0 = kb * 16 + 2 * kp;
            if (ga >= lines) continue;
            float2 xa[2], xb[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) split(k0 + e, pr, xa[e], xb[e]);
            const long long col = (long long)kb * kbstride + 2 * kp;
            gst<NTS>(reinterpret_cast<float4 *>(out + rowoff[2 * pr] + col), pack2(xa[0], xa[1]));
            if (ga + 1 < lines)
                gst<NTS>(reinterpret_cast<float4 *>(out + rowoff[2 * pr + 1] + col), pack2(xb[0], xb[1]));
            if (k0 == 0) {
                float2 na, nb;
                split(M, pr, na, nb);
                const long long cm = (long long)(NKB - 1) * kbstride;
                gst<NTS>(out + rowoff[2 * pr] + cm, na);
                if (ga + 1 < lines) gst<NTS>(out + rowoff[2 * pr + 1] + cm, nb);
            }
        }
        __syncthreads();  // LDS tile and row offsets are reused by the next tile
    }
};

template <int M, int MT, bool TR = false>
__global__ __launch_bounds__(M / 16 * 8) void k_r2c_p2(PassArgs a) {
    typedef R2cP2<M, MT, TR> K;
    __shared__ long long rowoff[16];
    float4 *buf = reinterpret_cast<float4 *>(pf_smem);
    K k(a, buf, reinterpret_cast<cx<float> *>(buf + M * K::CP), rowoff);
    k.init_tables(threadIdx.x, K::NT);
    int t = blockIdx.x;
    cx<float> p0[16], p1[16];
    if constexpr (MT != 0) {  // lanes of lines past the end compute on zeros
#pragma unroll
        for (int m = 0; m < 16; ++m) p0[m] = p1[m] = make_float2(0.f, 0.f);
    }
    if (t < k.ntiles) k.load(p0, p1, t, opaque_tid());
    __syncthreads();
    for (; t < k.ntiles; t += gridDim.x) {
        cx<float> v0[16], v1[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            v0[m] = p0[m];
            v1[m] = p1[m];
        }
        const int tn = t + gridDim.x;
        if (tn < k.ntiles) k.load(p0, p1, tn, opaque_tid());
        k.tile(v0, v1, t, opaque_tid());
    }
}

// The backward X stage split like R2cP2 (loads of one tile's spectra, inverse
// split, transform and stores of one tile).
template <int M, int MT, bool TR = false>
struct C2rP2 {
    static constexpr int TC = 16;
    static constexpr int T = M / 16;
    static constexpr int CP = 8;
    static constexpr int NT = T * CP;
    static constexpr int S = p2_stages(M);
    static constexpr int RL = p2_radix(M, S - 1);
    static constexpr int NSL = p2_ns(M, S - 1);
    static constexpr int NIT = M / 2 * 8 / NT;  // (mode k < M/2, line pair) items per thread per tile
    static_assert(NT % 128 == 0, "an item's line pair depends on tv only");
    static constexpr size_t kTileLds = (size_t)M * CP * 16;
    static constexpr size_t kTableLds = (size_t)(2 * M + 2) * 8 + (MT ? kMfmaTableBytes : 0);
    typedef typename MfmaSplit<MT == 0 ? 1 : MT>::vec avec;

    const PassArgs &a;
    float4 *buf;
    cx<float> *twl, *spl;
    avec *atab;  // matrix-core A operands (MT != 0)
    const cx<float> *__restrict__ in;
    float *__restrict__ out;
    int lines, ntiles;

    __device__ __forceinline__ C2rP2(const PassArgs &pa, float4 *tile_lds, cx<float> *tables) : a(pa) {
        buf = tile_lds;
        twl = tables;
        spl = twl + M;
        atab = reinterpret_cast<avec *>(twl + 2 * M + 2);
        in = reinterpret_cast<const cx<float> *>(a.in);
        out = reinterpret_cast<float *>(a.out);
        lines = (int)a.lines;
        ntiles = (lines + 15) / 16;
    }

    __device__ __forceinline__ void init_tables(int tv, int nthr) const {
        const cx<float> *__restrict__ tw = reinterpret_cast<const cx<float> *>(a.tw);
        for (int i = tv; i < 2 * M + 1; i += nthr)
            if (i != M - 1) twl[i] = tw[i];
        if constexpr (MT != 0) {
            if (tv < 64) {
                MfmaDft16<1, MT> d0;
                d0.init(tv);
                d0.store(atab, tv);
            }
        }
    }

    // item i of this thread: f = tv + NT i -> mode k = 16 kb + j (k < M/2) and line
    // pair pr; it holds X[k] and X[M-k] of both lines (for k = 0 the partner is
    // X[M], the first slot of the last column block), and threads 0..15 hold
    // X[M/2] of line tv.  A wave reads whole 128-byte rows of the workspace.
    // Addresses: one 64-bit tile base (uniform) plus offsets from it.
    // xk[2 i], xk[2 i + 1]: X[k] of the item's two lines; xm likewise X[M - k]
    __device__ __forceinline__ void load(cx<float> (&xk)[2 * NIT], cx<float> (&xm)[2 * NIT], float2 &xh, int t,
                                         int tv) const {
        if constexpr (TR) {
            // transposed rows: mode k of line g = z ny + y at z zrows + k kbrows + y
            // (zrows = nxh nyp, kbrows = nyp: 128-byte rows of 16 lines at one
            // mode).  The tile's 16 lines share a plane (ny is a multiple of 16).
            // Item f: line pair pr = f & 7 (8 lanes of 16 bytes along a row), mode
            // k = f >> 3 (k < M/2); it holds X[k] and X[M-k] of both lines, as the
            // blocked items do, and threads 0..15 hold X[M/2] of line tv.
            const int g0 = 16 * t;
            const int z0 = g0 / a.ny;
            const int y0 = g0 - z0 * a.ny;
            const cx<float> *tb = in + (long long)z0 * a.zrows + y0;
            const long long ks = a.kbrows;
#pragma unroll
            for (int i = 0; i < NIT; ++i) {
                const int f = tv + NT * i;
                const int pr = f & 7, k = f >> 3;
                const float4 u = gld<streamed<LD_C2R>()>(reinterpret_cast<const float4 *>(tb + k * ks + 2 * pr));
                const float4 w = gld<streamed<LD_C2R>()>(reinterpret_cast<const float4 *>(tb + (M - k) * ks + 2 * pr));
                xk[2 * i] = make_float2(u.x, u.y);
                xk[2 * i + 1] = make_float2(u.z, u.w);
                xm[2 * i] = make_float2(w.x, w.y);
                xm[2 * i + 1] = make_float2(w.z, w.w);
            }
            if (tv < 16) xh = gld<streamed<LD_C2R>()>(tb + (M / 2) * ks + tv);
            return;
        }
        const int g0 = 16 * t;
        const int z0 = g0 / a.ny;
        const int y0 = g0 - z0 * a.ny;
        const cx<float> *tb = in + (((long long)z0 * a.zrows + a.y0 + y0) << 4);
        const long long zplane = a.zrows * 16;  // elements between z planes of the workspace
        const long long kbs = a.kbrows * 16;    // elements between column blocks
        // line l of the tile (g = g0 + l, any number of z planes when ny < 16)
        // starts at row offset rowrel(l) from the tile base (z0, y0)
        auto rowrel = [&](int l) {
            const int g = g0 + l;
            const int z = g / a.ny;
            const int y = g - z * a.ny;
            return (long long)(z - z0) * zplane + (y - y0) * 16;
        };
        auto col = [&](int k) { return (long long)(k >> 4) * kbs + (k & 15); };
        // lines past the end load the last line instead; their results are never stored
        const int lmax = lines - 1 - g0;
        const int pr = (tv >> 4) & 7;  // the same line pair for every item (NT is a multiple of 128)
        const cx<float> *ra = tb + rowrel(min(2 * pr, lmax));
        const cx<float> *rb = tb + rowrel(min(2 * pr + 1, lmax));
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int f = tv + NT * i;
            const int k = ((f >> 7) << 4) + (f & 15);
            const int ck = col(k), cm = col(M - k);
            xk[2 * i] = gld<streamed<LD_C2R>()>(ra + ck);
            xm[2 * i] = gld<streamed<LD_C2R>()>(ra + cm);
            xk[2 * i + 1] = gld<streamed<LD_C2R>()>(rb + ck);
            xm[2 * i + 1] = gld<streamed<LD_C2R>()>(rb + cm);
        }
        if (tv < 16) xh = gld<streamed<LD_C2R>()>(tb + rowrel(min(tv, lmax)) + col(M / 2));
    }

    // Zb[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) W_nx^-k, one line
    __device__ __forceinline__ static float2 zb(float2 Xk, float2 Xm, float2 w) {
        const float2 E = make_float2(Xk.x + Xm.x, Xk.y - Xm.y);
        const float2 O = cmul(make_float2(Xk.x - Xm.x, Xk.y + Xm.y), w);
        return make_float2(E.x - O.y, E.y + O.x);
    }

    // inverse split from registers into LDS: item (k, pair) writes Zb[k] and
    // Zb[M-k] of both lines; modes 0 and M contribute their real parts only.
    // The caller synchronises before the transform reads the tile.
    __device__ __forceinline__ void split(const cx<float> (&pk)[2 * NIT], const cx<float> (&pm)[2 * NIT], float2 ph,
                                          int tv) const {
        {
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int f = tv + NT * i;
            // the item's mode and line pair (blocked or transposed rows, as in load())
            const int k = TR ? f >> 3 : ((f >> 7) << 4) + (f & 15);
            const int pr = TR ? f & 7 : (f >> 4) & 7;
            float2 Ak = pk[2 * i], Bk = pk[2 * i + 1];
            float2 Am = pm[2 * i], Bm = pm[2 * i + 1];
            if (k == 0) Ak.y = Bk.y = Am.y = Bm.y = 0.f;
            const cx<float> w = spl[k];
            const float2 wc = make_float2(w.x, -w.y);  // W_nx^-k
            buf[p2_slot<TC>(k, pr)] = pack2(zb(Ak, Am, wc), zb(Bk, Bm, wc));
            if (k != 0) {
                // Zb[M-k] uses W_nx^-(M-k) = -W_nx^k
                const float2 wm = make_float2(-w.x, -w.y);
                buf[p2_slot<TC>(M - k, pr)] = pack2(zb(Am, Ak, wm), zb(Bm, Bk, wm));
            }
        }
        }
        if (tv < 16) {
            const cx<float> w = spl[M / 2];
            reinterpret_cast<float2 *>(buf)[2 * p2_slot<TC>(M / 2, tv >> 1) + (tv & 1)] =
                zb(ph, ph, make_float2(w.x, -w.y));
        }
    }

    // The inverse transform of tile t (its spectra split into the LDS tile and
    // synchronised) and the stores of its real lines; ends with a barrier.
    __device__ __forceinline__ void tile(int t, int tv) const {
        const int cp_mid = tv % CP, q_mid = tv / CP;
        const int cp_out = tv / T, q_out = tv % T;
        cx<float> v0[16], v1[16];
        if constexpr (MT != 0) {  // stage 0 on the matrix cores, inputs from the LDS tile
            p2_stage0_mfma_lds<M, TC, 1, MT>(buf, atab, tv);
        } else {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            Dft<float, 16, 1>::run(v0);
            Dft<float, 16, 1>::run(v1);
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q_mid * 16 + r, cp_mid)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }
        if constexpr (S == 3 && MT != 0) {
            p2_stage1_mfma<M, TC, 1, MT>(buf, twl + p2_twoff(M, 1), atab, tv);
        } else if constexpr (S == 3) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            p2_butterflies2<M, 16, 16, 1>(v0, v1, q_mid, twl + p2_twoff(M, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(base + r * 16, cp_mid)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float4 x = buf[p2_slot<TC>(q_out + T * m, cp_out)];
            v0[m] = make_float2(x.x, x.y);
            v1[m] = make_float2(x.z, x.w);
        }
        p2_butterflies2<M, RL, NSL, 1>(v0, v1, q_out, twl + p2_twoff(M, S - 1));
        {
            const int ga = 16 * t + 2 * cp_out;
            float *oa = out + (long long)ga * a.ld_real + 2 * q_out;
            if (ga < lines) {
#pragma unroll
                for (int m = 0; m < 16; ++m) gst<streamed<ST_C2R>()>(reinterpret_cast<float2 *>(oa + 2 * T * m), v0[m]);
            }
            if (ga + 1 < lines) {
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    gst<streamed<ST_C2R>()>(reinterpret_cast<float2 *>(oa + a.ld_real + 2 * T * m), v1[m]);
            }
        }
        __syncthreads();
    }
};

template <int M, int MT, bool TR = false>
__global__ __launch_bounds__(M / 16 * 8, 2) void k_c2r_p2(PassArgs a) {
    typedef C2rP2<M, MT, TR> K;
    float4 *buf = reinterpret_cast<float4 *>(pf_smem);
    K k(a, buf, reinterpret_cast<cx<float> *>(buf + M * K::CP));
    k.init_tables(threadIdx.x, K::NT);
    int t = blockIdx.x;
    cx<float> pk[2 * K::NIT], pm[2 * K::NIT];
    float2 ph;
    if (t < k.ntiles) k.load(pk, pm, ph, t, threadIdx.x);
    __syncthreads();
    for (; t < k.ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        k.split(pk, pm, ph, tv);
        const int tn = t + gridDim.x;
        if (tn < k.ntiles) k.load(pk, pm, ph, tn, threadIdx.x);
        __syncthreads();
        k.tile(t, tv);
    }
}

// ---- X stage for power-of-two nx, FP64 ------------------------------------
// The FP32 X stage's method in double precision (Sec. 3.2): the real line x of
// length nx = 2M is transformed as the complex line z[m] = x[2m] + i x[2m+1]
// of length M and split into its M + 1 modes, X[k] = E[k] + W_nx^k O[k]; the
// backward pass inverts the split and runs the inverse DFT_M.  A tile is 8
// lines (16 on the transposed workspace), each a column of the FP64 C2C
// kernel's LDS map (one 16-byte slot per point and line); workspace rows hold
// 8 modes (128 bytes).  Twiddles as in
// FP32: the M-point stage table (M - 1 entries, copied to LDS), then at offset
// M the split table W_nx^k, k = 0 .. M, read from global memory (in LDS it
// would cost a block per CU at nx = 512).

// Row offset in the FP64 workspace of line g = z ny + y (8 modes per row).
__device__ __forceinline__ long long xd_rowoff(const PassArgs &a, int g) {
    const int z = g / a.ny;
    const int y = g - z * a.ny;
    return ((long long)z * a.zrows + a.y0 + y) << 3;
}

// TR: the spectra go to the transposed workspace (mode k of line g = z ny + y at
// z zrows + k kbrows + y, zrows = nxh ny, kbrows = ny, ny a multiple of 16): a
// tile is then 16 lines, so that one row holds 256 contiguous bytes per mode.
template <int M, bool TR = false>
__global__ __launch_bounds__(M / 16 * (TR ? 16 : 8)) void k_r2c_p2d(PassArgs a) {
    constexpr int TC = TR ? 16 : 8;  // lines per tile
    constexpr int T = M / 16;
    constexpr int NT = T * TC;
    constexpr int S = p2_stages(M);
    constexpr int RL = p2_radix(M, S - 1);
    constexpr int NSL = p2_ns(M, S - 1);
    constexpr int NKB = M / 8 + 1;  // column blocks of 8 modes for the M + 1 modes
    typedef cx<double> cd;
    __shared__ long long rowoff[TC];
    cd *buf = reinterpret_cast<cd *>(pf_smem);  // M points x TC lines
    cd *twl = buf + M * TC;                     // the stage table; the split table stays in global memory
    const cd *__restrict__ tw = reinterpret_cast<const cd *>(a.tw);
    const cd *__restrict__ spl = tw + M;
    for (int i = threadIdx.x; i < M - 1; i += NT) twl[i] = tw[i];
    const double *__restrict__ in = reinterpret_cast<const double *>(a.in);
    cd *__restrict__ out = reinterpret_cast<cd *>(a.out);
    const int lines = (int)a.lines;
    const int ntiles = (lines + TC - 1) / TC;
    const long long kbstride = a.kbrows << 3;
    auto slot = [](int p, int c) { return p2_slot<2 * TC>(p, c); };
    // line l = tv / T of tile t, points q + T m (lanes along the line)
    auto load = [&](cd(&d)[16], int t) {
        const int tv = opaque_tid();
        const int l = tv / T, q = tv % T;
        const int g = TC * t + l;
        if (g < lines) {
            const double *pl = in + (long long)g * a.ld_real + 2 * q;
#pragma unroll
            for (int m = 0; m < 16; ++m)
                d[m] = gld_d<streamed<LD_R2C>()>(reinterpret_cast<const double2 *>(pl + 2 * T * m));
        }
    };
    int t = blockIdx.x;
    cd p[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) p[m] = make_double2(0.0, 0.0);
    if (t < ntiles) load(p, t);
    __syncthreads();  // tables in LDS
    for (; t < ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        const int c_in = tv / T, q_in = tv % T;
        const int c_mid = tv % TC, q_mid = tv / TC;
        cd v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = p[m];
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(p, tn);
        if (!TR && tv < TC && TC * t + tv < lines) rowoff[tv] = xd_rowoff(a, TC * t + tv);
        Dft<double, 16, -1>::run(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[slot(q_in * 16 + r, c_in)] = v[r];
        __syncthreads();
        if constexpr (S == 3) {
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_mid + T * m, c_mid)];
            __syncthreads();
            p2_butterflies1<M, 16, 16, -1>(v, q_mid, twl + p2_twoff(M, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[slot(base + r * 16, c_mid)] = v[r];
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_mid + T * m, c_mid)];
        __syncthreads();
        p2_butterflies1<M, RL, NSL, -1>(v, q_mid, twl + p2_twoff(M, S - 1));
#pragma unroll
        for (int m = 0; m < 16; ++m) buf[slot(q_mid + T * m, c_mid)] = v[m];
        __syncthreads();
        // X[k] of line l from Z[k mod M] and Z[(M - k) mod M], k = 0 .. M
        auto split = [&](int k, int l) {
            const cd zk = buf[slot(k < M ? k : 0, l)];
            const cd zm = buf[slot((M - k) & (M - 1), l)];
            const cd E = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
            const cd O = make_double2(0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x));
            return cadd(E, cmul(spl[k], O));
        };
        if constexpr (TR) {
            // item f: line l = f & 15 (lanes along the row), mode k = f >> 4 < M; the
            // items of k = 0 also store mode M
            const int g0 = TC * t;
            const int z0 = g0 / a.ny;
            const int y0 = g0 - z0 * a.ny;
            cd *tb = out + (long long)z0 * a.zrows + y0;
            const int ks = (int)a.kbrows;
            for (int f = tv; f < M * TC; f += NT) {
                const int l = f & (TC - 1), k = f / TC;
                gst_d<streamed<ST_R2C>()>(reinterpret_cast<double2 *>(tb + (k * ks + l)), split(k, l));
                if (k == 0) gst_d<streamed<ST_R2C>()>(reinterpret_cast<double2 *>(tb + (M * ks + l)), split(M, l));
            }
            __syncthreads();  // the LDS tile is reused by the next tile
            continue;
        }
        // item f = (column block kb, line l, mode j): 8 lanes store one 128-byte row;
        // the items of k = 0 also store mode M, alone in the last column block
        for (int f = tv; f < (NKB - 1) * 64; f += NT) {
            const int kb = f >> 6, l = (f >> 3) & 7, j = f & 7;
            if (TC * t + l >= lines) continue;
            const int k = kb * 8 + j;
            cd *row = out + rowoff[l];
            gst_d<streamed<ST_R2C>()>(reinterpret_cast<double2 *>(row + kb * kbstride + j), split(k, l));
            if (k == 0)
                gst_d<streamed<ST_R2C>()>(reinterpret_cast<double2 *>(row + (NKB - 1) * kbstride), split(M, l));
        }
        __syncthreads();  // LDS tile and row offsets are reused by the next tile
    }
}

template <int M, bool TR = false>
__global__ __launch_bounds__(M / 16 * (TR ? 16 : 8)) void k_c2r_p2d(PassArgs a) {
    constexpr int TC = TR ? 16 : 8;  // lines per tile (TR: 256-byte transposed rows)
    constexpr int T = M / 16;
    constexpr int NT = T * TC;
    constexpr int S = p2_stages(M);
    constexpr int RL = p2_radix(M, S - 1);
    constexpr int NSL = p2_ns(M, S - 1);
    constexpr int NIT = M / 2 * TC / NT;  // (mode k < M/2, line) items per thread per tile
    static_assert(NT % 64 == 0, "an item's line depends on tv only");
    typedef cx<double> cd;
    cd *buf = reinterpret_cast<cd *>(pf_smem);
    cd *twl = buf + M * TC;  // the stage table; the split table stays in global memory
    const cd *__restrict__ tw = reinterpret_cast<const cd *>(a.tw);
    const cd *__restrict__ spl = tw + M;
    for (int i = threadIdx.x; i < M - 1; i += NT) twl[i] = tw[i];
    const cd *__restrict__ in = reinterpret_cast<const cd *>(a.in);
    double *__restrict__ out = reinterpret_cast<double *>(a.out);
    const int lines = (int)a.lines;
    const int ntiles = (lines + TC - 1) / TC;
    auto slot = [](int p, int c) { return p2_slot<2 * TC>(p, c); };
    // item i: f = tv + NT i -> mode k < M/2 of line l; it holds X[k] and X[M-k]
    // (for k = 0 the partner is X[M], the first slot of the last column
    // block), and threads 0..TC-1 hold X[M/2] of line tv.  A wave reads whole
    // rows.  Blocked rows (8 modes of one line): k = 8 (f >> 6) + (f & 7),
    // l = (f >> 3) & 7.  Transposed rows (TR: mode k of line g = z ny + y at
    // z zrows + k kbrows + y, zrows = nxh ny, kbrows = ny, so one 256-byte row
    // holds the tile's 16 lines at one mode; ny is a multiple of 16): l = f & 15,
    // k = f >> 4.
    auto item = [](int f, int &k, int &l) {
        if constexpr (TR) {
            l = f & (TC - 1);
            k = f / TC;
        } else {
            l = (f >> 3) & 7;
            k = ((f >> 6) << 3) + (f & 7);
        }
    };
    auto load = [&](cd(&xk)[NIT], cd(&xm)[NIT], cd &xh, int t, int tv) {
        const int g0 = TC * t;
        if constexpr (TR) {
            const int z0 = g0 / a.ny;
            const int y0 = g0 - z0 * a.ny;
            const cd *tb = in + (long long)z0 * a.zrows + y0;
            const long long ks = a.kbrows;
#pragma unroll
            for (int i = 0; i < NIT; ++i) {
                int k, l;
                item(tv + NT * i, k, l);
                xk[i] = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(tb + k * ks + l));
                xm[i] = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(tb + (M - k) * ks + l));
            }
            if (tv < TC) xh = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(tb + (M / 2) * ks + tv));
            return;
        }
        const int z0 = g0 / a.ny;
        const int y0 = g0 - z0 * a.ny;
        const cd *tb = in + (((long long)z0 * a.zrows + a.y0 + y0) << 3);
        const long long zplane = a.zrows * 8;  // elements between z planes of the workspace
        const long long kbs = a.kbrows * 8;    // elements between column blocks
        auto rowrel = [&](int l) {
            const int g = g0 + l;
            const int z = g / a.ny;
            const int y = g - z * a.ny;
            return (long long)(z - z0) * zplane + (y - y0) * 8;
        };
        auto col = [&](int k) { return (long long)(k >> 3) * kbs + (k & 7); };
        // lines past the end load the last line instead; their results are never stored
        const int lmax = lines - 1 - g0;
        const cd *r = tb + rowrel(min((tv >> 3) & 7, lmax));
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            int k, l;
            item(tv + NT * i, k, l);
            xk[i] = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(r + col(k)));
            xm[i] = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(r + col(M - k)));
        }
        if (tv < TC) xh = gld_d<streamed<LD_C2R>()>(reinterpret_cast<const double2 *>(tb + rowrel(min(tv, lmax)) + col(M / 2)));
    };
    // Zb[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) W_nx^-k
    auto zb = [](cd Xk, cd Xm, cd w) {
        const cd E = make_double2(Xk.x + Xm.x, Xk.y - Xm.y);
        const cd O = cmul(make_double2(Xk.x - Xm.x, Xk.y + Xm.y), w);
        return make_double2(E.x - O.y, E.y + O.x);
    };

    int t = blockIdx.x;
    cd pk[NIT], pm[NIT], ph = make_double2(0.0, 0.0);
    if (t < ntiles) load(pk, pm, ph, t, threadIdx.x);
    __syncthreads();  // tables in LDS
    for (; t < ntiles; t += gridDim.x) {
        const int tv = opaque_tid();
        // inverse split into the LDS tile; modes 0 and M contribute their real parts only
        {
#pragma unroll
            for (int i = 0; i < NIT; ++i) {
                int k, l;
                item(tv + NT * i, k, l);
                cd Xk = pk[i], Xm = pm[i];
                if (k == 0) Xk.y = Xm.y = 0.0;
                const cd w = spl[k];
                buf[slot(k, l)] = zb(Xk, Xm, make_double2(w.x, -w.y));
                // Zb[M-k] uses W_nx^-(M-k) = -W_nx^k
                if (k != 0) buf[slot(M - k, l)] = zb(Xm, Xk, make_double2(-w.x, -w.y));
            }
            if (tv < TC) {
                const cd w = spl[M / 2];
                buf[slot(M / 2, tv)] = zb(ph, ph, make_double2(w.x, -w.y));
            }
        }
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(pk, pm, ph, tn, tv);
        __syncthreads();
        const int c_mid = tv % TC, q_mid = tv / TC;
        const int c_out = tv / T, q_out = tv % T;
        cd v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_mid + T * m, c_mid)];
        __syncthreads();
        Dft<double, 16, 1>::run(v);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[slot(q_mid * 16 + r, c_mid)] = v[r];
        __syncthreads();
        if constexpr (S == 3) {
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_mid + T * m, c_mid)];
            __syncthreads();
            p2_butterflies1<M, 16, 16, 1>(v, q_mid, twl + p2_twoff(M, 1));
            const int k = q_mid & 15;
            const int base = (q_mid - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[slot(base + r * 16, c_mid)] = v[r];
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = buf[slot(q_out + T * m, c_out)];
        p2_butterflies1<M, RL, NSL, 1>(v, q_out, twl + p2_twoff(M, S - 1));
        const int g = TC * t + c_out;
        if (g < lines) {
            double *o = out + (long long)g * a.ld_real + 2 * q_out;
#pragma unroll
            for (int m = 0; m < 16; ++m) gst_d<streamed<ST_C2R>()>(reinterpret_cast<double2 *>(o + 2 * T * m), v[m]);
        }
        __syncthreads();  // the next tile's split overwrites the LDS tile
    }
}

// ---- fused X-Y pass: the slab form of the method (Sec. 4.3, Fig. 10) --------
// The X and Y stages of one z plane need no data from other planes, so one
// persistent kernel can run both, plane after plane, and the Y stage then
// reads the X stage's output of a plane shortly after it was written, while
// it can still be in the caches (one exchange instead of two, as in the
// paper's slab decomposition).  Work items: X tiles (producers) and Y tiles
// (consumers) of each plane, dealt to nq queues, one per XCD (plane z to
// queue z mod nq; a workgroup serves the queue of the XCD it runs on, read
// from the hardware), so that a plane's producers and consumers share one L2.
// Within a queue the items are ordered
//   X(P0) .. X(P(lag-1)), then X(P(j+lag)), Y(Pj) for j = 0, 1, ..., then the
//   remaining Y,
// and each block takes the next ticket of its queue.  A consumer item waits
// until every producer item of its plane has finished; those took earlier
// tickets of the same queue, so they are held by running blocks, and producer
// items never wait: the waits always end (no co-residency needed).  Each wait
// is also bounded (spin_limit polls); on expiry the status word is set, the
// item runs anyway and the host reports the timeout.  Hand-off: a producer's
// waves wait until their stores are complete (written to the XCD's L2; the
// L1 is write-through), then the item is counted with an atomic; a consumer
// polls the count and then loads the plane through the same L2.  No other
// work item reads those lines before (a tile's rows belong to one item), so
// no L1 holds a stale copy, and no L2 write-back or invalidation is needed.  The backward pass is the
// mirror: Y tiles (producers, sign +1), then the complex-to-real X tiles.
// The counters are zeroed by k_fused_reset before every launch.

// In-place Y tile on the blocked workspace (rows of 16 modes, 16 columns per
// tile, plain FP32): the k_c2c_p2 tile for two row sides, without its options.
template <int N, int DIR>
struct YRowsP2 {
    static constexpr int TC = 16;
    static constexpr int T = N / 16;
    static constexpr int CP = 8;
    static constexpr int NT = T * CP;
    static constexpr int S = p2_stages(N);
    static constexpr int RL = p2_radix(N, S - 1);
    static constexpr int NSL = p2_ns(N, S - 1);
    static constexpr size_t kTileLds = (size_t)N * CP * 16;
    static constexpr size_t kTableLds = (size_t)N * 8;
    float4 *buf;
    cx<float> *twl;
    cx<float> *ws;
    const cx<float> *tw;
    long long sa, sblk;  // workspace elements between z planes / column blocks
    int CB, C;

    __device__ __forceinline__ YRowsP2(const PassArgs &a, float4 *tile_lds, cx<float> *tables) {
        buf = tile_lds;
        twl = tables;
        ws = reinterpret_cast<cx<float> *>(a.out);
        tw = reinterpret_cast<const cx<float> *>(a.tw);
        sa = a.in_s.sa;
        sblk = a.in_s.sblk;
        CB = (int)a.CB;
        C = a.C;
    }
    __device__ __forceinline__ void init_tables(int tv, int nthr) const {
        for (int i = tv; i < N - 1; i += nthr) twl[i] = tw[i];
    }
    // element (column 2 cp, row 0) of tile t = (z, column block), valid columns
    __device__ __forceinline__ long long base(int t, int cp, int &ncol) const {
        const int z = t / CB, cb = t - z * CB;
        ncol = min(TC, C - cb * TC);
        return (long long)z * sa + (long long)cb * sblk + 2 * cp;
    }
    // live = false: a tile past the plane's last column block (no memory accesses)
    __device__ __forceinline__ void load(cx<float> (&d0)[16], cx<float> (&d1)[16], int t, int tv, bool live) const {
        const int cp = tv % CP, q = tv / CP;
        int ncol;
        const long long b = base(t, cp, ncol) + (long long)q * TC;
        if (live && 2 * cp < ncol) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = *reinterpret_cast<const float4 *>(ws + b + (long long)m * T * TC);
                d0[m] = make_float2(x.x, x.y);
                d1[m] = make_float2(x.z, x.w);
            }
        }
    }
    template <bool NTS>
    __device__ __forceinline__ void tile(cx<float> (&v0)[16], cx<float> (&v1)[16], int t, int tv, bool live) const {
        const int cp = tv % CP, q = tv / CP;
        Dft<float, 16, DIR>::run(v0);
        Dft<float, 16, DIR>::run(v1);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q * 16 + r, cp)] = pack2(v0[r], v1[r]);
        __syncthreads();
        if constexpr (S == 3) {
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q + T * m, cp)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            p2_butterflies2<N, 16, 16, DIR>(v0, v1, q, twl + p2_twoff(N, 1));
            const int k = q & 15;
            const int bse = (q - k) * 16 + k;
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(bse + r * 16, cp)] = pack2(v0[r], v1[r]);
            __syncthreads();
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const float4 x = buf[p2_slot<TC>(q + T * m, cp)];
            v0[m] = make_float2(x.x, x.y);
            v1[m] = make_float2(x.z, x.w);
        }
        p2_butterflies2<N, RL, NSL, DIR>(v0, v1, q, twl + p2_twoff(N, S - 1));
        int ncol;
        const long long b = base(t, cp, ncol) + (long long)q * TC;
        if (live && 2 * cp < ncol) {
#pragma unroll
            for (int m = 0; m < 16; ++m)
                gst<NTS>(reinterpret_cast<float4 *>(ws + b + (long long)m * T * TC), pack2(v0[m], v1[m]));
        }
        __syncthreads();  // the next item reuses the LDS tile
    }
};

// s_getreg_b32 operand for the XCC_ID hardware register (id 20, bits 0..3):
// the XCD a workgroup runs on
constexpr int kHwRegXccId = (3 << 11) | 20;
// s_waitcnt operand that waits for every vector memory access of the wave
// (vmcnt 0; expcnt and lgkmcnt left at their maxima)
constexpr int kWaitVmcnt0 = 0x0F70;

// Counters of one fused launch: [0, nq) queue tickets, [nq, nq + nz) finished
// producer items per plane; the status word after them is left alone.
__global__ __launch_bounds__(256) void k_fused_reset(unsigned *ctl, int n) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) ctl[i] = 0u;
}

// Forward (FWD = 1): X stage (R2cP2<M>) then Y stage (sign -1) per plane.
// Backward (FWD = 0): Y stage (sign +1) then X stage (C2rP2<M>).  A block has
// 512 threads; an X item is XT = 512 / (M/2) tiles of 16 lines run side by
// side, a Y item YT = 512 / (NY/2) tiles (z, column block).
template <int M, int NY, int FWD>
__global__ __launch_bounds__(512) void k_xy_fused(FusedArgs f) {
    typedef R2cP2<M, 0> XF;
    typedef C2rP2<M, 0> XB;
    typedef YRowsP2<NY, FWD ? -1 : 1> Y;
    constexpr int XNT = XF::NT, XT = 512 / XNT;
    constexpr int YT = 512 / Y::NT;
    static_assert(XT * XNT == 512 && YT * Y::NT == 512 && XB::NT == XNT, "items fill the block");
    static_assert(2 * XB::NIT == 16, "the backward X loads fit the item registers");
    constexpr size_t XAREA = XT * XF::kTileLds, YAREA = YT * Y::kTileLds;
    constexpr size_t AREA = XAREA > YAREA ? XAREA : YAREA;
    __shared__ long long rowoff[XT][16];
    __shared__ int s_item[4];  // kind, plane, index, next item's loads issued early
    unsigned char *lds = pf_smem;
    cx<float> *xtab = reinterpret_cast<cx<float> *>(lds + AREA);
    cx<float> *ytab = reinterpret_cast<cx<float> *>(lds + AREA + XF::kTableLds);
    const int tid = threadIdx.x;
    const int xh = tid / XNT, yh = tid / Y::NT;  // X / Y tile of the item the thread works on
    float4 *xbuf = reinterpret_cast<float4 *>(lds + xh * XF::kTileLds);
    float4 *ybuf = reinterpret_cast<float4 *>(lds + yh * Y::kTileLds);
    const XF xf(f.x, xbuf, xtab, rowoff[xh]);
    const XB xb(f.x, xbuf, xtab);
    const Y yk(f.y, ybuf, ytab);
    if constexpr (FWD) xf.init_tables(tid, 512);
    else xb.init_tables(tid, 512);
    yk.init_tables(tid, 512);

    // the block's queue is its XCD: producer and consumer items of a plane then
    // share one L2, which holds the producers' stores once they are complete,
    // so the hand-off needs no cache write-back or invalidation
    const int q = (int)(__builtin_amdgcn_s_getreg(kHwRegXccId) & 15u);
    if (q >= f.nq) return;  // no XCD beyond the queues the host found (its plan would be refused)
    const int np = (f.nz - q + f.nq - 1) / f.nq;  // planes q, q + nq, ... of this queue
    unsigned *tickets = f.ctl;
    unsigned *done = f.ctl + f.nq;
    unsigned *status = f.ctl + f.nq + f.nz;
    const int pitems = FWD ? f.xitems : f.yitems;  // producer / consumer items per plane
    const int citems = FWD ? f.yitems : f.xitems;
    const int xall = f.nz * f.xtiles, yall = f.nz * f.ytiles;  // tiles of the X / Y stage

    // thread 0: take the next ticket of the queue and decode it into s_item
    // (kind -1 past the end)
    auto fetch = [&]() {
        if (tid == 0) {
            const int k = (int)__hip_atomic_fetch_add(tickets + q, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int kind = -1, j = 0, idx = 0;
            if (!fused_item(k, np, f.lag, pitems, citems, kind, j, idx)) kind = -1;
            s_item[0] = kind;
            s_item[1] = q + j * f.nq;
            s_item[2] = idx;
        }
    };
    // thread 0: has every producer item of the plane finished?  With wait, poll
    // until it has (bounded: past spin_limit polls the status word is set)
    auto ready = [&](int plane, bool wait) -> bool {
        unsigned *c = done + plane;
        long long polls = 0;
        while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)pitems) {
            if (!wait) return false;
            if (++polls > f.spin_limit) {
                __hip_atomic_fetch_or(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        return true;
    };
    auto is_x = [](int kind) { return (kind == 0) == (FWD != 0); };
    // this thread's tile of an item, and whether it exists (the plane's last
    // item may be partly empty)
    auto item_tile = [&](int kind, int plane, int idx, bool &live) {
        if (is_x(kind)) {
            const int r = idx * XT + xh;
            live = r < f.xtiles;
            return live ? plane * f.xtiles + r : xall;
        }
        const int r = idx * YT + yh;
        live = r < f.ytiles;
        return live ? plane * f.ytiles + r : yall;
    };
    cx<float> p0[16], p1[16];  // loads of the next item
    float2 ph = make_float2(0.f, 0.f);
#pragma unroll
    for (int m = 0; m < 16; ++m) p0[m] = p1[m] = make_float2(0.f, 0.f);
    // thread indices are re-derived per use from an opaque copy of threadIdx.x:
    // held across the item loop, the LDS addresses built from them would not
    // fit the registers
    auto load = [&](int kind, int plane, int idx) {
        const int tv = opaque_tid();
        bool live;
        const int t = item_tile(kind, plane, idx, live);
        if (is_x(kind)) {
            if (live) {
                if constexpr (FWD) xf.load(p0, p1, t, tv % XNT);
                else xb.load(p0, p1, ph, t, tv % XNT);
            }
        } else {
            yk.load(p0, p1, t, tv % Y::NT, live);
        }
    };

    fetch();
    __syncthreads();  // tables in LDS, first item in s_item
    int kind = s_item[0], plane = s_item[1], idx = s_item[2];
    if (kind == 1 && tid == 0) ready(plane, true);
    __syncthreads();
    if (kind >= 0) load(kind, plane, idx);
    while (kind >= 0) {
        cx<float> v0[16], v1[16];
        const float2 vh = ph;
#pragma unroll
        for (int m = 0; m < 16; ++m) v0[m] = p0[m], v1[m] = p1[m];
        // the next item: its loads go out now if it is a producer or its plane is complete
        __syncthreads();  // every thread has read s_item
        fetch();
        __syncthreads();
        const int nkind = s_item[0], nplane = s_item[1], nidx = s_item[2];
        if (tid == 0) s_item[3] = nkind == 0 ? 1 : (nkind == 1 && ready(nplane, false) ? 1 : 0);
        __syncthreads();
        const bool early = nkind >= 0 && s_item[3];
        if (early) load(nkind, nplane, nidx);
        // the current item
        const int tv = opaque_tid();
        bool live;
        const int t = item_tile(kind, plane, idx, live);
        if (is_x(kind)) {
            if constexpr (FWD) {
                xf.template tile<false>(v0, v1, t, tv % XNT);  // t past the end stores nothing
            } else {
                xb.split(v0, v1, vh, tv % XNT);
                __syncthreads();
                xb.tile(t, tv % XNT);
            }
        } else {
            // plain stores: with the nontemporal hint here the compiler keeps the
            // tile's registers in scratch memory
            yk.template tile<false>(v0, v1, t, tv % Y::NT, live);
        }
        if (kind == 0) {  // a producer item: its stores complete (in the L2), then publish it
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(done + plane, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        kind = nkind, plane = nplane, idx = nidx;
        if (kind >= 0 && !early) {
            if (kind == 1 && tid == 0) ready(plane, true);
            __syncthreads();
            load(kind, plane, idx);
        }
    }
}

// nx: 1024 or 2048 (X half length 512 / 1024); ny: 512 or 1024
bool p2_fused_supported(int nx, int ny, int prec) {
    return prec == 0 && (nx == 1024 || nx == 2048) && (ny == 512 || ny == 1024);
}

template <int M, int NY>
static constexpr size_t fused_lds() {
    constexpr size_t xa = (512 / R2cP2<M, 0>::NT) * R2cP2<M, 0>::kTileLds;
    constexpr size_t ya = (512 / YRowsP2<NY, 1>::NT) * YRowsP2<NY, 1>::kTileLds;
    return (xa > ya ? xa : ya) + R2cP2<M, 0>::kTableLds + YRowsP2<NY, 1>::kTableLds;
}

size_t p2_fused_lds_bytes(int nx, int ny) {
    if (nx == 1024) return ny == 512 ? fused_lds<512, 512>() : fused_lds<512, 1024>();
    return ny == 512 ? fused_lds<1024, 512>() : fused_lds<1024, 1024>();
}

int p2_fused_tiles_per_item(int n, int x) { return x ? 512 / (n / 2 / 16 * 8) : 512 / (n / 16 * 8); }

static const void *fused_pick(int nx, int ny, int fwd) {
#define PF_FUSED_PICK(NXV, NYV)                                                                       \
    if (nx == NXV && ny == NYV)                                                                       \
        return fwd ? (const void *)&k_xy_fused<NXV / 2, NYV, 1> : (const void *)&k_xy_fused<NXV / 2, NYV, 0>;
    PF_FUSED_PICK(1024, 512)
    PF_FUSED_PICK(1024, 1024)
    PF_FUSED_PICK(2048, 512)
    PF_FUSED_PICK(2048, 1024)
#undef PF_FUSED_PICK
    return nullptr;
}

const void *p2_fused_symbol(int nx, int ny, int fwd) { return fused_pick(nx, ny, fwd); }

// XCD of every workgroup of a launch of `blocks` workgroups
__global__ __launch_bounds__(64) void k_xcc_probe(unsigned *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg(kHwRegXccId) & 15u;
}

hipError_t p2_xcd_queues(unsigned blocks, int *nq) {
    *nq = 0;
    unsigned *d = nullptr;
    hipError_t e = hipMalloc(&d, blocks * sizeof(unsigned));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xcc_probe, dim3(blocks), dim3(64), 0, 0, d);
    std::vector<unsigned> h(blocks);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(h.data(), d, blocks * sizeof(unsigned), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return e;
    unsigned seen = 0;
    for (unsigned v : h) seen |= 1u << v;
    int n = 0;
    while (n < 16 && (seen >> n) & 1u) ++n;
    if (n > 0 && seen == (1u << n) - 1u) *nq = n;  // XCDs 0 .. n-1, each with workgroups
    return hipSuccess;
}

hipError_t p2_fused_prepare(int nx, int ny) {
    for (int fwd : {0, 1}) {
        const void *k = fused_pick(nx, ny, fwd);
        if (!k) return hipErrorInvalidValue;
        const hipError_t e =
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p2_fused_lds_bytes(nx, ny));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t p2_fused_launch(const FusedArgs &f, int fwd, int nx, int ny, unsigned blocks, hipStream_t s) {
    const void *k = fused_pick(nx, ny, fwd);
    if (!k) return hipErrorInvalidDeviceFunction;
    const int n = f.nq + f.nz;
    hipLaunchKernelGGL(k_fused_reset, dim3((n + 255) / 256), dim3(256), 0, s, f.ctl, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    FusedArgs a = f;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(blocks), dim3(512), args, p2_fused_lds_bytes(nx, ny), s);
}

bool p2x_supported(int nx, int prec) {
    return (prec == 0 && (nx == 512 || nx == 1024 || nx == 2048)) || (prec == 1 && (nx == 512 || nx == 1024));
}

int p2x_threads(int nx, int prec, int tr) { return nx / 2 / 16 * (prec == 1 && tr ? 16 : 8); }

int p2x_tile_lines(int prec, int tr) { return prec == 1 && !tr ? 8 : 16; }

size_t p2x_lds_bytes(int nx, int math, int prec, int tr) {
    const int M = nx / 2;
    if (prec == 1) return (size_t)M * p2x_tile_lines(1, tr) * sizeof(double2) + (size_t)M * sizeof(double2);
    return (size_t)M * 16 * sizeof(float2) + (size_t)(2 * M + 2) * sizeof(float2) + (math ? kMfmaTableBytes : 0);
}

static const void *p2xd_pick(int nx, int fwd, int tr = 0) {
    if (nx == 512)
        return fwd ? (tr ? (const void *)&k_r2c_p2d<256, true> : (const void *)&k_r2c_p2d<256>)
                   : (tr ? (const void *)&k_c2r_p2d<256, true> : (const void *)&k_c2r_p2d<256>);
    if (nx == 1024)
        return fwd ? (tr ? (const void *)&k_r2c_p2d<512, true> : (const void *)&k_r2c_p2d<512>)
                   : (tr ? (const void *)&k_c2r_p2d<512, true> : (const void *)&k_c2r_p2d<512>);
    return nullptr;
}

static const void *p2x_pick(int nx, int fwd, int mt, int tr = 0) {
#define PF_X_PICK(NXV, MV)                                                                    \
    if (nx == NXV) {                                                                          \
        if (tr && mt != 0) return nullptr;                                                    \
        if (tr) return fwd ? (const void *)&k_r2c_p2<MV, 0, true> : (const void *)&k_c2r_p2<MV, 0, true>; \
        if (mt == 0) return fwd ? (const void *)&k_r2c_p2<MV, 0> : (const void *)&k_c2r_p2<MV, 0>; \
        if (MV < 512) return nullptr;                                                         \
        if (mt == 1) return fwd ? (const void *)&k_r2c_p2<MV, MV < 512 ? 0 : 1>               \
                                : (const void *)&k_c2r_p2<MV, MV < 512 ? 0 : 1>;              \
        return fwd ? (const void *)&k_r2c_p2<MV, MV < 512 ? 0 : 2> : (const void *)&k_c2r_p2<MV, MV < 512 ? 0 : 2>; \
    }
    PF_X_PICK(512, 256)
    PF_X_PICK(1024, 512)
    PF_X_PICK(2048, 1024)
#undef PF_X_PICK
    return nullptr;
}

hipError_t p2x_prepare(int nx, int prec) {
    hipError_t e = hipSuccess;
    if (prec == 1) {
        for (int v = 0; v < 4; ++v) {  // (forward, transposed rows) = (v & 1, v >> 1)
            const void *k = p2xd_pick(nx, v & 1, v >> 1);
            if (!k) return hipErrorInvalidValue;
            const hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)p2x_lds_bytes(nx, 0, 1, v >> 1));
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    for (int fwd : {0, 1})
        for (int mt = 0; mt < 4; ++mt) {  // mt 3: the transposed-row kernels (plain)
        const void *k = mt < 3 ? p2x_pick(nx, fwd, mt) : p2x_pick(nx, fwd, 0, 1);
        if (!k) continue;
        hipError_t r =
            hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p2x_lds_bytes(nx, mt < 3 ? mt : 0, 0, 0));
        if (r != hipSuccess && e == hipSuccess) e = r;
        }
    return e;
}

int p2_tc(int n) { return n <= 1024 ? 16 : 16384 / n; }

size_t p2_lds_bytes(int n, int math) {
    return ((size_t)n * p2_tc(n) + n) * sizeof(float2) + (math == 1 || math == 2 ? kMfmaTableBytes : 0);
}

bool p2_supported(int n, int prec) {
    return prec == 0 && (n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096);
}

bool p2d_supported(int n) { return n == 256 || n == 512 || n == 1024; }
size_t p2d_lds_bytes(int n) { return (size_t)n * 8 * 16 + (size_t)n * 16; }
int p2d_threads(int n) { return n / 16 * 8; }

template <int N, int DIR>
static const void *p2d_pick_dir(int inp, int outp) {
    if (inp == 0 && outp == 0) return reinterpret_cast<const void *>(&k_c2c_p2d<N, DIR, 0, 0>);
    if (inp == 0 && outp == 1) return reinterpret_cast<const void *>(&k_c2c_p2d<N, DIR, 0, 1>);
    if (inp == 1 && outp == 0) return reinterpret_cast<const void *>(&k_c2c_p2d<N, DIR, 1, 0>);
    // lines on both sides: the Y passes of the transposed chains
    if (inp == 1 && outp == 1) return reinterpret_cast<const void *>(&k_c2c_p2d<N, DIR, 1, 1>);
    return nullptr;
}

static const void *p2d_pick(int n, int dir, int inp, int outp) {
    switch (n) {
        case 256: return dir < 0 ? p2d_pick_dir<256, -1>(inp, outp) : p2d_pick_dir<256, 1>(inp, outp);
        case 512: return dir < 0 ? p2d_pick_dir<512, -1>(inp, outp) : p2d_pick_dir<512, 1>(inp, outp);
        case 1024: return dir < 0 ? p2d_pick_dir<1024, -1>(inp, outp) : p2d_pick_dir<1024, 1>(inp, outp);
        default: return nullptr;
    }
}

hipError_t p2d_prepare(int n) {
    for (int dir : {-1, 1})
        for (int io = 0; io < 4; ++io) {  // (inp, outp): (0,0) (0,1) (1,0) (1,1)
            const void *k = p2d_pick(n, dir, io >= 2 ? 1 : 0, io & 1);
            if (!k) return hipErrorInvalidValue;
            const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p2d_lds_bytes(n));
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

template <int N, int TC, int DIR, int INP, int OUTP, int MT>
static const void *p2_kernel() {
    return reinterpret_cast<const void *>(&k_c2c_p2<N, TC, DIR, INP, OUTP, MT>);
}

template <int N, int TC, int DIR, int MT>
static const void *p2_pick_io_dir(int inp, int outp) {
    if (inp == 0 && outp == 0) return p2_kernel<N, TC, DIR, 0, 0, MT>();
    if (inp == 0 && outp == 1) return p2_kernel<N, TC, DIR, 0, 1, MT>();
    if (inp == 1 && outp == 0) return p2_kernel<N, TC, DIR, 1, 0, MT>();
    if (inp == 0 && outp == 2) return p2_kernel<N, TC, DIR, 0, 2, MT>();
    if (inp == 2 && outp == 0) return p2_kernel<N, TC, DIR, 2, 0, MT>();
    if constexpr (MT == 0) {  // lines in place: the Y passes on the transposed workspace
        if (inp == 1 && outp == 1) return p2_kernel<N, TC, DIR, 1, 1, MT>();
    }
    return nullptr;
}

template <int N, int TC, int MT>
static const void *p2_pick_io(int dir, int inp, int outp) {
    return dir < 0 ? p2_pick_io_dir<N, TC, -1, MT>(inp, outp) : p2_pick_io_dir<N, TC, 1, MT>(inp, outp);
}

// kernel symbol for (n, dir, inp, outp, math); nullptr if not built.  The
// matrix-core variants exist for the 16-column tiles with a middle radix-16
// stage: n = 512 and 1024.
// mt: 0 plain, 1 / 2 matrix-core middle stage (512 and 1024 only), 3 no
// transform, 4 type-I DCT by the even extension
static const void *p2_pick(int n, int dir, int inp, int outp, int mt) {
    switch (n) {
        case 256:
            return mt == 0 ? p2_pick_io<256, 16, 0>(dir, inp, outp)
                 : mt == 3 ? p2_pick_io<256, 16, 3>(dir, inp, outp)
                 : mt == 4 ? p2_pick_io<256, 16, 4>(dir, inp, outp) : nullptr;
        case 512:
            return mt == 0 ? p2_pick_io<512, 16, 0>(dir, inp, outp)
                 : mt == 1 ? p2_pick_io<512, 16, 1>(dir, inp, outp)
                 : mt == 2 ? p2_pick_io<512, 16, 2>(dir, inp, outp)
                 : mt == 3 ? p2_pick_io<512, 16, 3>(dir, inp, outp)
                           : p2_pick_io<512, 16, 4>(dir, inp, outp);
        case 1024:
            return mt == 0 ? p2_pick_io<1024, 16, 0>(dir, inp, outp)
                 : mt == 1 ? p2_pick_io<1024, 16, 1>(dir, inp, outp)
                 : mt == 2 ? p2_pick_io<1024, 16, 2>(dir, inp, outp)
                 : mt == 3 ? p2_pick_io<1024, 16, 3>(dir, inp, outp)
                           : p2_pick_io<1024, 16, 4>(dir, inp, outp);
        case 2048:
            return mt == 0 ? p2_pick_io<2048, 8, 0>(dir, inp, outp)
                 : mt == 3 ? p2_pick_io<2048, 8, 3>(dir, inp, outp)
                 : mt == 4 ? p2_pick_io<2048, 8, 4>(dir, inp, outp) : nullptr;
        case 4096:
            return mt == 0 ? p2_pick_io<4096, 4, 0>(dir, inp, outp)
                 : mt == 3 ? p2_pick_io<4096, 4, 3>(dir, inp, outp)
                 : mt == 4 ? p2_pick_io<4096, 4, 4>(dir, inp, outp) : nullptr;
        default: return nullptr;
    }
}

const void *p2_symbol(const PassDesc &d) {
    if (d.kind == PASS_C2C_P2 && d.prec == 1) return p2d_pick(d.a.fft.n, d.dir, d.a.inp, d.a.outp);
    if (d.kind == PASS_R2C_P2)
        return d.prec == 1 ? p2xd_pick(2 * d.a.fft.n, 1, d.a.xtr) : p2x_pick(2 * d.a.fft.n, 1, d.a.math, d.a.xtr);
    if (d.kind == PASS_C2R_P2)
        return d.prec == 1 ? p2xd_pick(2 * d.a.fft.n, 0, d.a.xtr) : p2x_pick(2 * d.a.fft.n, 0, d.a.math, d.a.xtr);
    return p2_pick(d.a.fft.n, d.dir, d.a.inp, d.a.outp, d.a.math);
}

template <int N, int TC>
static const void *spec_pick_n(int adj) {
    return adj ? reinterpret_cast<const void *>(&k_spec_p2<N, TC, 1>)
               : reinterpret_cast<const void *>(&k_spec_p2<N, TC, 0>);
}

// fused spectral-step kernel for extension length n; nullptr if not built
static const void *spec_pick(int n, int adj) {
    switch (n) {
        case 256: return spec_pick_n<256, 16>(adj);
        case 512: return spec_pick_n<512, 16>(adj);
        case 1024: return spec_pick_n<1024, 16>(adj);
        case 2048: return spec_pick_n<2048, 8>(adj);
        case 4096: return spec_pick_n<4096, 4>(adj);
        default: return nullptr;
    }
}

hipError_t p2_spec_prepare(int n) {
    for (int adj = 0; adj < 2; ++adj) {
        const void *k = spec_pick(n, adj);
        if (!k) return hipErrorInvalidValue;
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p2_lds_bytes(n, 0));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int p2_spec_blocks_per_cu(int n, unsigned threads, size_t lds) {
    int nb = 0;
    const void *k = spec_pick(n, 0);
    if (!k) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)threads, lds) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

#ifndef PF_SPEC_SR
#define PF_SPEC_SR 1  // 0: the fused spectral step keeps the even extension at nz = 257 too
#endif
bool p2_spec_sr_supported(int nz) { return PF_SPEC_SR && nz == 257; }
unsigned p2_spec_sr_threads(int nz) { return nz == 257 ? 256 / 16 * 8 + 256 / 32 * 8 : 0; }
size_t p2_spec_sr_lds_bytes(int nz) {
    const int L = nz - 1, M = L / 2;
    return (size_t)(L + M) * 8 * sizeof(float4) + (size_t)(L + 2 * M) * sizeof(float2);
}

hipError_t p2_spec_launch(const PassDesc &d, int adj, int nx, float scale, hipStream_t s) {
    const void *k = d.a.math == 5 && d.a.cheb == 257
                        ? (adj ? (const void *)&k_spec_sr<256, 1> : (const void *)&k_spec_sr<256, 0>)
                        : spec_pick(d.a.fft.n, adj);
    if (!k) return hipErrorInvalidDeviceFunction;
    PassArgs a = d.a;
    void *args[] = {&a, &nx, &scale};
    return hipLaunchKernel(k, dim3(d.blocks), dim3(d.threads), args, d.lds, s);
}

bool p2_has_mfma(int n) { return n == 512 || n == 1024; }

hipError_t p2_prepare(int n) {
    hipError_t e = hipSuccess;
    for (int dir : {-1, 1})
        for (int io = 0; io < 30; ++io) {
            const int mt = io / 6, k6 = io % 6;  // (inp, outp): (0,0) (0,1) (1,0) (0,2) (2,0) (1,1)
            const int inp = k6 == 2 || k6 == 5 ? 1 : k6 == 4 ? 2 : 0, outp = k6 == 1 || k6 == 5 ? 1 : k6 == 3 ? 2 : 0;
            const void *k = p2_pick(n, dir, inp, outp, mt);
            if (!k) continue;
            hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p2_lds_bytes(n, mt));
            if (r != hipSuccess && e == hipSuccess) e = r;
        }
    return e;
}

int p2_blocks_per_cu(const PassDesc &d) {
    int nb = 0;
    const void *k = p2_symbol(d);
    if (!k) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)d.threads, d.lds) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

int p2_threads(int n) { return n / 16 * p2_tc(n) / 2; }

hipError_t p2_launch(const PassDesc &d, hipStream_t s) {
    const void *k = p2_symbol(d);
    if (!k) return hipErrorInvalidDeviceFunction;
    PassArgs a = d.a;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(d.blocks), dim3(d.threads), args, d.lds, s);
}

}  // namespace pf
