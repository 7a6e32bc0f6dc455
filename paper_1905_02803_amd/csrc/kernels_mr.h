// kernels_mr.h -- FP32 passes for mixed-radix lengths with the plan fixed at
// compile time (the Y / Z column passes and the X real-line passes of the
// transpose-based 3D FFT, Sec. 2).
//
// A length N = N1 N2 (N1 <= N2 <= 36, every factor 2, 3, 5 or 7) is done in
// two Cooley-Tukey steps with input index n = q + N2 m and output index
// k = k1 + N1 k2 (q, k2 < N2; m, k1 < N1):
//     Y[q][k1]          = W_N^{q k1} sum_m x[q + N2 m] W_N1^{m k1}      (step 1)
//     X[k1 + N1 k2]     = sum_q Y[q][k1] W_N2^{q k2}                    (step 2)
// Each step is one in-register DFT per thread whose radix structure and
// internal twiddles are compile-time constants; the only exchange between
// threads is the LDS tile between the steps.  A C2C tile (16 columns of one
// 128-byte workspace row block) reads its step-1 inputs straight from global
// memory into registers and stores the step-2 outputs straight from
// registers: one LDS round trip per tile, against one per radix stage plus
// the staging of the load and the store in the runtime-radix kernels.
// Lanes run along the 16 columns of the tile on both sides.
//
// The X passes carry two real lines as one complex line (a + i b), as the
// runtime-radix X kernels do; their loads and stores run along the points of
// the lines, and the real/complex split (forward) or the Hermitian fill
// (backward) goes through LDS.
#pragma once

#include "fft_device.h"
#include "pf_internal.h"

namespace pf {

extern __shared__ __align__(16) unsigned char pf_smem[];

// ---- cos / sin of 2 pi m / n, evaluated by the compiler -----------------------
// The angle is reduced exactly in integers to a quarter turn plus an angle in
// [0, pi/2), folded to [0, pi/4] by the complement, and summed by its Taylor
// series (13 terms: truncation below 1e-25 there).
__host__ __device__ constexpr double ct_sin_series(double x) {
    double term = x, sum = x;
    for (int i = 1; i <= 12; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr double ct_cos_series(double x) {
    double term = 1.0, sum = 1.0;
    for (int i = 1; i <= 12; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}
__host__ __device__ constexpr double ct_trig(int m, int n, bool want_sin) {
    const long long r = ((long long)m % n + n) % n;
    const long long q = (4 * r) / n;     // quarter turns
    const long long rr = 4 * r - q * n;  // rest: (pi / 2) rr / n
    const bool flip = 2 * rr > n;
    const double x = 1.57079632679489661923 * (double)(flip ? n - rr : rr) / (double)n;
    const double s0 = flip ? ct_cos_series(x) : ct_sin_series(x);
    const double c0 = flip ? ct_sin_series(x) : ct_cos_series(x);
    const double c = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
    const double s = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
    return want_sin ? s : c;
}

// ---- in-register DFT of any 7-smooth size (natural order in and out) ----------
// Sizes 2, 3, 4, 5, 7, 8, 16 use the fixed kernels; any other N = A B runs B
// DFTs of size A over x[B n1 + n2], twiddles by W_N^{n2 k1}, and A DFTs of size
// B, output k1 + A k2.
template <int N>
struct MrSplit {
    static constexpr int A = (N % 16 == 0 && N > 16) ? 16
                           : (N % 8 == 0 && N > 8)   ? 8
                           : (N % 4 == 0 && N > 4)   ? 4
                           : (N % 2 == 0)            ? 2
                           : (N % 3 == 0)            ? 3
                           : (N % 5 == 0)            ? 5
                                                     : 7;
    static constexpr int B = N / A;
};

template <int N, int DIR>
struct DftMR {
    __device__ __forceinline__ static void run(cx<float> *v) {
        if constexpr (N == 1) {
        } else if constexpr (N == 2 || N == 3 || N == 4 || N == 5 || N == 7 || N == 8 || N == 16) {
            Dft<float, N, DIR>::run(v);
        } else {
            constexpr int A = MrSplit<N>::A, B = MrSplit<N>::B;
            static_assert(A * B == N && B > 1, "size must be 7-smooth");
            cx<float> t[B][A];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
                for (int n1 = 0; n1 < A; ++n1) t[n2][n1] = v[B * n1 + n2];
                DftMR<A, DIR>::run(t[n2]);
            }
#pragma unroll
            for (int n2 = 1; n2 < B; ++n2)
#pragma unroll
                for (int k1 = 1; k1 < A; ++k1)
                    t[n2][k1] = crot<DIR>(t[n2][k1], (float)ct_trig(n2 * k1, N, false), (float)ct_trig(n2 * k1, N, true));
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) {
                cx<float> u[B];
#pragma unroll
                for (int n2 = 0; n2 < B; ++n2) u[n2] = t[n2][k1];
                DftMR<B, DIR>::run(u);
#pragma unroll
                for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k2];
            }
        }
    }
};

// ---- tile geometry -----------------------------------------------------------
#ifndef PF_MR_SPZ_RES
#define PF_MR_SPZ_RES 2
#endif
// X kernels: line pairs per tile (a power of two; the lines' workspace rows are
// separate, so the tile width does not change the row accesses)
#ifndef PF_MR_XP
#define PF_MR_XP 4
#endif
// C2C kernel: two step-1 items per thread for strongly unbalanced factor pairs
#ifndef PF_MR_HALF
#define PF_MR_HALF 1
#endif
// global accesses with the nontemporal hint: bit 0 stores, bit 1 loads
#ifndef PF_MR_NT
#define PF_MR_NT 0
#endif
typedef float mr_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 mr_ld(const float2 *p) {
    if constexpr ((PF_MR_NT & 2) != 0) {
        const mr_f2 u = __builtin_nontemporal_load(reinterpret_cast<const mr_f2 *>(p));
        return make_float2(u.x, u.y);
    } else {
        return *p;
    }
}
__device__ __forceinline__ float mr_ld(const float *p) {
    if constexpr ((PF_MR_NT & 2) != 0) return __builtin_nontemporal_load(p);
    else return *p;
}
__device__ __forceinline__ void mr_st(float2 *p, float2 v) {
    if constexpr ((PF_MR_NT & 1) != 0) {
        const mr_f2 u = {v.x, v.y};
        __builtin_nontemporal_store(u, reinterpret_cast<mr_f2 *>(p));
    } else {
        *p = v;
    }
}
__device__ __forceinline__ void mr_st(float *p, float v) {
    if constexpr ((PF_MR_NT & 1) != 0) __builtin_nontemporal_store(v, p);
    else *p = v;
}

__host__ __device__ constexpr int mr_threads(int n1, int n2) {
    return 16 * (((n1 > n2 ? n1 : n2) + 3) / 4 * 4);  // 16 columns x max(N1, N2) items, whole waves
}
// Threads per column of the C2C kernel: max(N1, N2) rounded up to 4, or, where
// N2 >= 2 N1 and N2 >= 24, max(N1, ceil(N2 / 2)) with up to two step-1 items
// per thread -- smaller workgroups, of which more fit on a CU, where step 2
// would leave most threads idle.  Measured per length on the Y pass: faster
// for N2 of 25 and more (lengths 125, 175, 243, 250; 245 even), slower by
// 4-8% for N2 of 21 and less.
__host__ __device__ constexpr int mr_c2c_cols(int n1, int n2) {
    const int full = ((n1 > n2 ? n1 : n2) + 3) / 4 * 4;
    const int half2 = (n2 + 1) / 2;
    const int half = ((n1 > half2 ? n1 : half2) + 3) / 4 * 4;
    return PF_MR_HALF && n2 >= 2 * n1 && n2 >= 24 && half < full ? half : full;
}
__host__ __device__ constexpr int mr_c2c_threads(int n1, int n2) { return 16 * mr_c2c_cols(n1, n2); }
// X kernels: PF_MR_XP pairs x max(N1, N2) items, whole waves
__host__ __device__ constexpr int mr_x_threads(int n1, int n2) {
    return (PF_MR_XP * (n1 > n2 ? n1 : n2) + 63) / 64 * 64;
}

template <int N1, int N2>
struct MrShape {
    static constexpr int N = N1 * N2;
    static constexpr int NQ = N1 > N2 ? N1 : N2;
    static constexpr int THREADS = mr_threads(N1, N2);
    // exchange tile: row (c, k1) or (k1, c) of P2 entries, P2 odd so that the
    // step-2 reads of consecutive rows fall on different banks
    static constexpr int P2 = N2 % 2 == 0 ? N2 + 1 : N2;
    static constexpr int XCH = 16 * N1 * P2;
    // X passes: XP line pairs per tile, XTHREADS threads; one complex line per
    // pair at pitch SP (= 16 mod 32, >= N)
    static constexpr int XP = PF_MR_XP;
    static constexpr int XTHREADS = mr_x_threads(N1, N2);
    static constexpr int SP = N + ((16 - N % 32) % 32 + 32) % 32;
    static constexpr int XLDS = XP * N1 * P2 > XP * SP ? XP * N1 * P2 : XP * SP;
    // C2C pass with a line side: line-major tile copy at pitch SPZ (= PF_MR_SPZ_RES
    // mod 32, >= N), written and read by lanes along the columns
    static constexpr int SPZ = N + ((PF_MR_SPZ_RES - N % 32) % 32 + 32) % 32;
    static constexpr int CLDS = XCH > 16 * SPZ ? XCH : 16 * SPZ;
    // C2C kernel: threads per column, threads, step-1 items per thread
    static constexpr int CT = mr_c2c_cols(N1, N2);
    static constexpr int CTHREADS = 16 * CT;
    static constexpr int I1 = (N2 + CT - 1) / CT;
};

// ---- C2C column tile -----------------------------------------------------------
struct MrC2C {
    const cx<float> *in;
    cx<float> *out;
    const cx<float> *tw;  // W_N^m, m < N (forward sign)
    long long ib, isc, isp, ob, osc, osp;
    int ncol;
};

__device__ __forceinline__ long long mr_side_base(const Side &s, long long a, int cb) {
    const int cpb = (int)s.cpb;
    const int blk = cb / cpb;
    return a * s.sa + (long long)blk * s.sblk + (long long)((cb - blk * cpb) * 16) * s.sc;
}

// tile `tile` of the C2C pass a (16 columns per tile), reading inp, writing outp
__device__ __forceinline__ MrC2C mr_c2c_args(const PassArgs &a, const void *inp, void *outp, long long tile) {
    MrC2C t;
    // tile order 1 walks the outer index fastest (neighbouring tiles then touch
    // adjacent rows and lines of sides whose column blocks lie far apart)
    const int CB = (int)a.CB, A = (int)a.A;
    const int ta = a.tile_order ? (int)tile % A : (int)tile / CB;
    const int cb = a.tile_order ? (int)tile / A : (int)tile - ta * CB;
    t.in = reinterpret_cast<const cx<float> *>(inp);
    t.out = reinterpret_cast<cx<float> *>(outp);
    t.tw = reinterpret_cast<const cx<float> *>(a.tw);
    t.ib = mr_side_base(a.in_s, ta, cb);
    t.ob = mr_side_base(a.out_s, ta, cb);
    t.isc = a.in_s.sc, t.isp = a.in_s.sp, t.osc = a.out_s.sc, t.osp = a.out_s.sp;
    const int left = a.C - cb * 16;
    t.ncol = left < 16 ? left : 16;
    return t;
}

template <int N1, int N2, int DIR>
__device__ __forceinline__ void mr_c2c_body(const MrC2C &t) {
    using S = MrShape<N1, N2>;
    constexpr int N = S::N;
    constexpr int NT = S::CTHREADS;
    constexpr int ITEMS = (16 * N + NT - 1) / NT;  // tile points per thread
    cx<float> *lds = reinterpret_cast<cx<float> *>(pf_smem);
    const int tid = threadIdx.x;
    const int c = tid & 15, j = tid >> 4;
    const bool cv = c < t.ncol;
    // a side whose columns are whole lines (points contiguous) goes through a
    // line-major LDS copy of the tile, so that its global accesses run along
    // the points; a row side is read / written by the step-1 / step-2 threads
    const bool in_lines = t.isp == 1 && t.isc != 1;
    const bool out_lines = t.osp == 1 && t.osc != 1;
    if (in_lines) {
        cx<float> r[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int f = tid + i * NT;
            const int cc = f / N, p = f - cc * N;
            r[i] = make_float2(0.f, 0.f);
            if (f < 16 * N && cc < t.ncol) r[i] = mr_ld(t.in + t.ib + cc * t.isc + p);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int f = tid + i * NT;
            const int cc = f / N, p = f - cc * N;
            if (f < 16 * N) lds[cc * S::SPZ + p] = r[i];
        }
        __syncthreads();
    }
    // step 1, items q = j + it CT (it < I1): the N1 points q + N2 m of column c;
    // every item's loads are issued before the first transform
    cx<float> x[S::I1][N1];
#pragma unroll
    for (int it = 0; it < S::I1; ++it) {
        const int q = j + it * S::CT;
#pragma unroll
        for (int m = 0; m < N1; ++m) x[it][m] = make_float2(0.f, 0.f);
        if (q < N2) {
            if (in_lines) {
#pragma unroll
                for (int m = 0; m < N1; ++m) x[it][m] = lds[c * S::SPZ + q + N2 * m];
            } else if (cv) {
                const cx<float> *src = t.in + t.ib + c * t.isc + q * t.isp;
                const long long step = (long long)N2 * t.isp;
#pragma unroll
                for (int m = 0; m < N1; ++m) x[it][m] = mr_ld(src + m * step);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < S::I1; ++it) {
        const int q = j + it * S::CT;
        if (q < N2) {
            DftMR<N1, DIR>::run(x[it]);
#pragma unroll
            for (int k1 = 1; k1 < N1; ++k1) {
                cx<float> w = t.tw[q * k1];
                if (DIR > 0) w.y = -w.y;
                x[it][k1] = cmul(x[it][k1], w);
            }
        }
    }
    if (in_lines) __syncthreads();  // the staged lines are read before the exchange tile overwrites them
#pragma unroll
    for (int it = 0; it < S::I1; ++it) {
        const int q = j + it * S::CT;
        if (q < N2) {
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1) lds[(k1 * S::P2 + q) * 16 + c] = x[it][k1];
        }
    }
    __syncthreads();
    cx<float> y[N2];
    if (j < N1) {  // step 2, item k1 = j: outputs k1 + N1 k2 of column c
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) y[n2] = lds[(j * S::P2 + n2) * 16 + c];
        DftMR<N2, DIR>::run(y);
    }
    if (out_lines) {
        __syncthreads();  // the exchange tile is read before the line-major copy overwrites it
        if (j < N1) {
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) lds[c * S::SPZ + j + N1 * k2] = y[k2];
        }
        __syncthreads();
        cx<float> r[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int f = tid + i * NT;
            const int cc = f / N, p = f - cc * N;
            if (f < 16 * N) r[i] = lds[cc * S::SPZ + p];
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int f = tid + i * NT;
            const int cc = f / N, p = f - cc * N;
            if (f < 16 * N && cc < t.ncol) mr_st(t.out + t.ob + cc * t.osc + p, r[i]);
        }
    } else if (j < N1 && cv) {
        cx<float> *dst = t.out + t.ob + c * t.osc + j * t.osp;
        const long long step = (long long)N1 * t.osp;
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) mr_st(dst + k2 * step, y[k2]);
    }
}

// ---- X passes: PF_MR_XP pairs of real lines per tile ----------------------------
struct MrX {
    const void *in;
    void *out;
    const cx<float> *tw;  // W_N^m, m < N = nx (forward sign)
    long long g0, lines, ld_real, ny, zrows, kbstride;
    int y0, nkb, nxh;
};

__device__ __forceinline__ MrX mr_x_args(const PassArgs &a, const void *inp, void *outp, long long tile) {
    MrX t;
    t.in = inp;
    t.out = outp;
    t.tw = reinterpret_cast<const cx<float> *>(a.tw);
    t.g0 = tile * (2 * PF_MR_XP);
    t.lines = a.lines;
    t.ld_real = a.ld_real;
    t.ny = a.ny;
    t.zrows = a.zrows;
    t.kbstride = a.kbrows << 4;
    t.y0 = a.y0;
    t.nkb = a.nkb;
    t.nxh = a.nxh;
    return t;
}

// row offset (workspace, column block 0) of the 2 PF_MR_XP lines of the tile:
// line g = z ny + y starts at row z zrows + y0 + y
__device__ __forceinline__ void mr_rowoff(const MrX &t, long long *rowoff) {
    const int tid = threadIdx.x;
    if (tid < 2 * PF_MR_XP) {
        const long long g = t.g0 + tid;
        const long long z = g / t.ny;
        const long long y = g - z * t.ny;
        rowoff[tid] = (z * t.zrows + t.y0 + y) << 4;
    }
}

// forward: real lines -> half spectra in the blocked workspace
template <int N1, int N2>
__device__ __forceinline__ void mr_r2c_body(const MrX &t) {
    using S = MrShape<N1, N2>;
    constexpr int N = S::N;
    __shared__ long long rowoff[2 * PF_MR_XP];
    cx<float> *lds = reinterpret_cast<cx<float> *>(pf_smem);
    const int tid = threadIdx.x;
    mr_rowoff(t, rowoff);
    const float *__restrict__ in = reinterpret_cast<const float *>(t.in);
    cx<float> *__restrict__ out = reinterpret_cast<cx<float> *>(t.out);
    if (tid < S::XP * N2) {  // step 1, item (c, q): lanes along the points of the lines
        const int c = tid / N2, q = tid - c * N2;
        const long long ga = t.g0 + 2 * c;
        cx<float> x[N1];
#pragma unroll
        for (int m = 0; m < N1; ++m) x[m] = make_float2(0.f, 0.f);
        if (ga < t.lines) {
            const float *pa = in + ga * t.ld_real + q;
#pragma unroll
            for (int m = 0; m < N1; ++m) x[m].x = mr_ld(pa + N2 * m);
        }
        if (ga + 1 < t.lines) {
            const float *pb = in + (ga + 1) * t.ld_real + q;
#pragma unroll
            for (int m = 0; m < N1; ++m) x[m].y = mr_ld(pb + N2 * m);
        }
        DftMR<N1, -1>::run(x);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) x[k1] = cmul(x[k1], t.tw[q * k1]);
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) lds[(c * N1 + k1) * S::P2 + q] = x[k1];
    }
    __syncthreads();
    cx<float> y[N2];
    const int c2 = tid / N1, k1 = tid - c2 * N1;
    if (tid < S::XP * N1) {  // step 2, item (c, k1)
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) y[n2] = lds[(c2 * N1 + k1) * S::P2 + n2];
        DftMR<N2, -1>::run(y);
    }
    __syncthreads();  // the exchange tile is read before the spectra overwrite it
    if (tid < S::XP * N1) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) lds[c2 * S::SP + k1 + N1 * k2] = y[k2];
    }
    __syncthreads();
    // split Z = A + i B into the half spectra of the two lines, row by row:
    // mode (kb, cc, kk), lanes along the 16 modes of a row
    const int total = t.nkb * 16 * S::XP;
    for (int f = tid; f < total; f += S::XTHREADS) {
        const int kk = f & 15, cc = (f >> 4) & (S::XP - 1), kb = f / (16 * S::XP);
        const int k = kb * 16 + kk;
        const long long ga = t.g0 + 2 * cc;
        if (k < t.nxh && ga < t.lines) {
            const cx<float> z = lds[cc * S::SP + k];
            const cx<float> w = lds[cc * S::SP + (k == 0 ? 0 : N - k)];
            const long long o = kb * t.kbstride + kk;
            mr_st(out + rowoff[2 * cc] + o, make_float2((z.x + w.x) * 0.5f, (z.y - w.y) * 0.5f));
            if (ga + 1 < t.lines) mr_st(out + rowoff[2 * cc + 1] + o, make_float2((z.y + w.y) * 0.5f, (w.x - z.x) * 0.5f));
        }
    }
}

// backward: half spectra in the blocked workspace -> real lines
template <int N1, int N2>
__device__ __forceinline__ void mr_c2r_body(const MrX &t) {
    using S = MrShape<N1, N2>;
    constexpr int N = S::N;
    constexpr int EH = 4;  // rows in flight per thread before the LDS writes
    __shared__ long long rowoff[2 * PF_MR_XP];
    cx<float> *lds = reinterpret_cast<cx<float> *>(pf_smem);
    const int tid = threadIdx.x;
    mr_rowoff(t, rowoff);
    __syncthreads();
    const cx<float> *__restrict__ in = reinterpret_cast<const cx<float> *>(t.in);
    float *__restrict__ out = reinterpret_cast<float *>(t.out);
    // Z = A + i B on the whole line: modes k < nxh from the rows, the rest by
    // Hermitian symmetry; the imaginary parts of modes 0 and N / 2 are dropped
    const int total = t.nkb * 16 * S::XP;
    for (int f1 = tid; f1 < total; f1 += EH * S::XTHREADS) {
        cx<float> ra[EH], rb[EH];
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            ra[i] = rb[i] = make_float2(0.f, 0.f);
            const int f = f1 + i * S::XTHREADS;
            const int kk = f & 15, cc = (f >> 4) & (S::XP - 1), kb = f / (16 * S::XP);
            const int k = kb * 16 + kk;
            const long long ga = t.g0 + 2 * cc;
            if (f < total && k < t.nxh && ga < t.lines) {
                const long long o = kb * t.kbstride + kk;
                ra[i] = mr_ld(in + rowoff[2 * cc] + o);
                if (ga + 1 < t.lines) rb[i] = mr_ld(in + rowoff[2 * cc + 1] + o);
            }
        }
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int f = f1 + i * S::XTHREADS;
            const int kk = f & 15, cc = (f >> 4) & (S::XP - 1), kb = f / (16 * S::XP);
            const int k = kb * 16 + kk;
            if (f < total && k < t.nxh) {
                const cx<float> A = ra[i], B = rb[i];
                cx<float> *col = lds + cc * S::SP;
                if (k == 0 || 2 * k == N) {
                    col[k] = make_float2(A.x, B.x);
                } else {
                    col[k] = make_float2(A.x - B.y, A.y + B.x);
                    col[N - k] = make_float2(A.x + B.y, B.x - A.y);
                }
            }
        }
    }
    __syncthreads();
    const int c = tid / N2, q = tid - c * N2;
    cx<float> x[N1];
    if (tid < S::XP * N2) {  // step 1, item (c, q)
#pragma unroll
        for (int m = 0; m < N1; ++m) x[m] = lds[c * S::SP + q + N2 * m];
        DftMR<N1, 1>::run(x);
#pragma unroll
        for (int k1 = 1; k1 < N1; ++k1) {
            cx<float> w = t.tw[q * k1];
            w.y = -w.y;
            x[k1] = cmul(x[k1], w);
        }
    }
    __syncthreads();  // the lines are read before the exchange tile overwrites them
    if (tid < S::XP * N2) {
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) lds[(c * N1 + k1) * S::P2 + q] = x[k1];
    }
    __syncthreads();
    if (tid < S::XP * N1) {  // step 2, item (c, k1): real parts to line 2c, imaginary to 2c + 1
        const int c2 = tid / N1, k1 = tid - c2 * N1;
        cx<float> y[N2];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) y[n2] = lds[(c2 * N1 + k1) * S::P2 + n2];
        DftMR<N2, 1>::run(y);
        const long long ga = t.g0 + 2 * c2;
        if (ga < t.lines) {
            float *pa = out + ga * t.ld_real + k1;
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) mr_st(pa + N1 * k2, y[k2].x);
        }
        if (ga + 1 < t.lines) {
            float *pb = out + (ga + 1) * t.ld_real + k1;
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) mr_st(pb + N1 * k2, y[k2].y);
        }
    }
}

// ---- kernels: one tile per workgroup, a plan's pass or a batch's ------------------
// MrArgs.b.count == 0: the plan's pass arguments `one`; else the batch work
// list b (transforms of this one length).
struct MrArgs {
    PassArgs one;
    BatchArgs b;
};

__device__ __forceinline__ int mr_find(const BatchArgs &b, long long blk) {
    int lo = 0, hi = b.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.first[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int N1, int N2, int DIR>
__global__ __launch_bounds__(mr_c2c_threads(N1, N2)) void k_mr_c2c(MrArgs m) {
    const long long blk = blockIdx.x;
    MrC2C t;
    if (m.b.count == 0) {
        t = mr_c2c_args(m.one, m.one.in, m.one.out, blk);
    } else {
        const int i = mr_find(m.b, blk);
        const PassArgs &a = m.b.args[i];
        t = mr_c2c_args(a, m.b.in_user ? (const void *)(m.b.user_in + (size_t)a.in) : a.in,
                        m.b.out_user ? (void *)(m.b.user_out + (size_t)a.out) : a.out, blk - m.b.first[i]);
    }
    mr_c2c_body<N1, N2, DIR>(t);
}

template <int N1, int N2, int FWD>
__global__ __launch_bounds__(mr_x_threads(N1, N2)) void k_mr_x(MrArgs m) {
    const long long blk = blockIdx.x;
    MrX t;
    if (m.b.count == 0) {
        t = mr_x_args(m.one, m.one.in, m.one.out, blk);
    } else {
        const int i = mr_find(m.b, blk);
        const PassArgs &a = m.b.args[i];
        t = mr_x_args(a, m.b.in_user ? (const void *)(m.b.user_in + (size_t)a.in) : a.in,
                      m.b.out_user ? (void *)(m.b.user_out + (size_t)a.out) : a.out, blk - m.b.first[i]);
    }
    if constexpr (FWD) mr_r2c_body<N1, N2>(t);
    else mr_c2r_body<N1, N2>(t);
}

// Lengths with a compile-time plan: X(N, N1, N2), N1 <= N2 the factor pair
// closest to sqrt(N).  Every 7-smooth length from 48 to 320 but 256 (a
// power-of-two kernel's), and 360, 480.  Four lists, one per compilation
// unit (kernels_mr_p0.hip .. p3), dealt round-robin so the units take about
// the same time to build.
#define PF_MR_LENGTHS_0(X) \
    X(48, 6, 8) X(56, 7, 8) X(70, 7, 10) X(81, 9, 9) X(98, 7, 14) X(112, 8, 14) X(128, 8, 16) \
    X(147, 7, 21) X(168, 12, 14) X(192, 12, 16) X(216, 12, 18) X(243, 9, 27) X(270, 15, 18) \
    X(300, 15, 20) X(480, 20, 24)
#define PF_MR_LENGTHS_1(X) \
    X(49, 7, 7) X(60, 6, 10) X(72, 8, 9) X(84, 7, 12) X(100, 10, 10) X(120, 10, 12) X(135, 9, 15) \
    X(150, 10, 15) X(175, 7, 25) X(196, 14, 14) X(224, 14, 16) X(245, 7, 35) X(280, 14, 20) \
    X(315, 15, 21)
#define PF_MR_LENGTHS_2(X) \
    X(50, 5, 10) X(63, 7, 9) X(75, 5, 15) X(90, 9, 10) X(105, 7, 15) X(125, 5, 25) X(140, 10, 14) \
    X(160, 10, 16) X(180, 12, 15) X(200, 10, 20) X(225, 15, 15) X(250, 10, 25) X(288, 16, 18) \
    X(320, 16, 20)
#define PF_MR_LENGTHS_3(X) \
    X(54, 6, 9) X(64, 8, 8) X(80, 8, 10) X(96, 8, 12) X(108, 9, 12) X(126, 9, 14) X(144, 12, 12) \
    X(162, 9, 18) X(189, 9, 21) X(210, 14, 15) X(240, 15, 16) X(252, 14, 18) X(294, 14, 21) \
    X(360, 18, 20)
#define PF_MR_LENGTHS(X) PF_MR_LENGTHS_0(X) PF_MR_LENGTHS_1(X) PF_MR_LENGTHS_2(X) PF_MR_LENGTHS_3(X)

// kernel of the length-N1 N2 passes: what = 0 forward C2C, 1 backward C2C,
// 2 forward X (real to half spectra), 3 backward X
template <int N1, int N2>
const void *mr_kernel_of(int what) {
    static_assert(MrShape<N1, N2>::XLDS * 8 + 2 * PF_MR_XP * 8 <= 65536 && MrShape<N1, N2>::CLDS * 8 <= 65536,
                  "tile within the default dynamic LDS limit");
    switch (what) {
        case 0: return reinterpret_cast<const void *>(&k_mr_c2c<N1, N2, -1>);
        case 1: return reinterpret_cast<const void *>(&k_mr_c2c<N1, N2, 1>);
        case 2: return reinterpret_cast<const void *>(&k_mr_x<N1, N2, 1>);
        case 3: return reinterpret_cast<const void *>(&k_mr_x<N1, N2, 0>);
    }
    return nullptr;
}
const void *mr_kernel_p0(int n, int what);
const void *mr_kernel_p1(int n, int what);
const void *mr_kernel_p2(int n, int what);
const void *mr_kernel_p3(int n, int what);

}  // namespace pf
