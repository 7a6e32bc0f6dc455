// kernels.hip -- transform kernels of the pencil 3D R2C / C2R FFT for gfx950.
//
// Each kernel is one HBM pass of the transpose-based 3D FFT (Sec. 2, Fig. 2):
// a workgroup loads a tile of whole lines of the axis being transformed into
// LDS, runs a mixed-radix Stockham FFT on every line of the tile, and writes
// the tile back.  The re-orientation between pencils (the paper's pack,
// all-to-all and unpack, Sec. 3.3) is folded into the address maps of these
// loads and stores, so each stage reads and writes the array exactly once.
//
//  k_r2c_x  : X stage of the forward transform.  Two real lines a, b are
//             packed as one complex line z = a + i b, transformed together,
//             and separated with A[k] = (Z[k] + conj Z[n-k]) / 2,
//             B[k] = (Z[k] - conj Z[n-k]) / (2 i), keeping k <= n/2 (the
//             (Nx+2)/2 modes of Sec. 3.2).
//  k_c2r_x  : X stage of the backward transform: the inverse of the above,
//             using only Re of modes 0 and n/2 (the modes Sec. 3.2 states are
//             real) and the conjugate-symmetric extension for the rest.
//  k_c2c_tile: C2C along Y or Z for a tile of TC adjacent columns; columns
//             are contiguous in memory so every row of the tile is one
//             coalesced segment, and the output may be laid out differently
//             from the input (the fused transpose).
#include "fft_device.h"
#include "pf_internal.h"

namespace pf {

extern __shared__ __align__(16) unsigned char pf_smem[];

// Twiddle tables are read through a pointer qualified as global memory: the
// stage functions below are out of line, and an unqualified pointer would
// turn every access into a flat one (as would a pointer into LDS, which is
// why the stages take the column as an element offset into pf_smem).
#define PF_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ cx<T> load_tw(const PF_GLOBAL cx<T> *p) {
    const PF_GLOBAL T *q = reinterpret_cast<const PF_GLOBAL T *>(p);
    return cmk<T>(q[0], q[1]);
}

// ---- one Stockham stage on one LDS column ------------------------------
// Butterfly j (j < n/R) reads x[j + r n/R], applies W_{Ns R}^{r k} with
// k = j mod Ns, runs the radix-R DFT and writes (j - k) R + k + r Ns.
// Every thread of the workgroup must call this (it holds two barriers).
// Kept out of line: inlining all radices into the runtime stage loop makes
// the register allocator keep their live ranges together.  The column is
// pf_smem element col_off on (so that its accesses are LDS instructions);
// j mod Ns is j - floor(j mag / 2^32) Ns with mag = ceil(2^32 / Ns), exact
// for j, Ns < 2^16.
template <typename T>
struct EMax {
    static constexpr int value = sizeof(T) == 4 ? kEMax : kEMax / 2;
};
// global accesses a thread keeps in flight when it moves a tile between HBM
// and LDS (FP64: fewer, so that the staging registers do not spill)
template <typename T>
struct Stage {
    static constexpr int value = sizeof(T) == 4 ? 16 : 4;
};

template <typename T, int R, int DIR>
__device__ __attribute__((noinline)) void fft_stage(int col_off, int n, int Ns, unsigned mag,
                                                    const PF_GLOBAL cx<T> *__restrict__ tw, int lane, int wpc) {
    constexpr int BM = (EMax<T>::value + R - 1) / R;
    cx<T> *col = reinterpret_cast<cx<T> *>(pf_smem) + col_off;
    const int nb = n / R;
    cx<T> v[BM][R];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const int j = lane + i * wpc;
        if (j < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = col[pidx(j + r * nb)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BM; ++i) {
        const int j = lane + i * wpc;
        if (j < nb) {
            const int k = Ns > 1 ? j - (int)__umulhi((unsigned)j, mag) * Ns : 0;
            if (Ns > 1) {
                const PF_GLOBAL cx<T> *t = tw + k * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = load_tw<T>(t + r - 1);
                    if (DIR > 0) w.y = -w.y;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            Dft<T, R, DIR>::run(v[i]);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) col[pidx(base + r * Ns)] = v[i][r];
        }
    }
    __syncthreads();
}

// Whole 1D FFT of length fs.n on the LDS column at pf_smem element col_off,
// in natural order.
template <typename T, int DIR>
__device__ __forceinline__ void fft_lds(int col_off, const FftSpec &fs, const cx<T> *tw_table, int lane, int wpc) {
    const PF_GLOBAL cx<T> *tw = (const PF_GLOBAL cx<T> *)tw_table;
    int Ns = 1;
    for (int s = 0; s < fs.nstages; ++s) {
        const int R = fs.radix[s];
        const PF_GLOBAL cx<T> *t = tw + fs.twoff[s];
        const unsigned mag = Ns > 1 ? 0xFFFFFFFFu / (unsigned)Ns + 1u : 0u;
        switch (R) {
            case 16: fft_stage<T, 16, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            case 8: fft_stage<T, 8, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            case 4: fft_stage<T, 4, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            case 2: fft_stage<T, 2, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            case 3: fft_stage<T, 3, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            case 5: fft_stage<T, 5, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
            default: fft_stage<T, 7, DIR>(col_off, fs.n, Ns, mag, t, lane, wpc); break;
        }
        Ns *= R;
    }
}

__device__ __forceinline__ long long side_base(const Side &s, int a, int cb, int tc) {
    const int cpb = (int)s.cpb;
    const int blk = cb / cpb;
    return (long long)a * s.sa + (long long)blk * s.sblk + (long long)((cb - blk * cpb) * tc) * s.sc;
}

// ---- C2C along a strided axis, TC columns per workgroup -------------------
// Tile `tile` of the pass a, reading `inp` and writing `outp` (the pass's own
// buffers, or the batch's).  The workgroup may have more threads than the
// tile's TC x wpc (a batched launch sized for its largest transform): the
// surplus threads help with the loads and stores and sit out the stages.
template <typename T, int DIR>
__device__ __forceinline__ void c2c_tile_body(const PassArgs &a, const void *inp, void *outp, long long tile) {
    cx<T> *lds = reinterpret_cast<cx<T> *>(pf_smem);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int TC = 1 << a.tc_log2;
    const int wpc = 1 << a.wpc_log2;
    // tile counts stay below 2^31 (checked at plan time): 32-bit index arithmetic
    const int CB = (int)a.CB;
    const int ta = (int)tile / CB;
    const int cb = (int)tile - ta * CB;
    const long long ib = side_base(a.in_s, ta, cb, TC);
    const long long ob = side_base(a.out_s, ta, cb, TC);
    const int left = a.C - cb * TC;
    const int ncol = left < TC ? left : TC;
    const int n = a.fft.n;
    const int pitch = a.pitch;
    const cx<T> *__restrict__ in = reinterpret_cast<const cx<T> *>(inp);
    cx<T> *__restrict__ out = reinterpret_cast<cx<T> *>(outp);
    const int rows_per = (nthr >> a.tc_log2) > 0 ? (nthr >> a.tc_log2) : 1;

    // type-I DCT (a.cheb > 0): point p of the even extension is source point p or n - p
    const int cheb = a.cheb;
    auto src = [cheb, n](int p) { return cheb > 0 && p >= cheb ? n - p : p; };
    // per thread: column c, points p0, p0 + dp, ...; element (c, p) at base + p sp
    const bool in_rows = a.in_s.sc == 1;  // rows of the tile contiguous: column fastest
    {
        const int c = in_rows ? (tid & (TC - 1)) : (tid >> a.wpc_log2);
        const int p0 = in_rows ? (tid >> a.tc_log2) : (tid & (wpc - 1));
        const int dp = in_rows ? rows_per : wpc;
        const long long sp = a.in_s.sp;
        const cx<T> *base = in + ib + (long long)c * a.in_s.sc;
        cx<T> *dst = lds + c * pitch;
        if (c < ncol) {
            // EM loads in flight before the first wait, then the LDS writes
            constexpr int EM = Stage<T>::value;
            const long long step = (long long)dp * sp;
            for (int p1 = p0; p1 < n; p1 += EM * dp) {
                // zeroed first: with only the in-range entries written the compiler
                // kept the FP64 array in scratch memory
                cx<T> r[EM];
#pragma unroll
                for (int i = 0; i < EM; ++i) r[i] = cmk<T>(T(0), T(0));
                const cx<T> *q = base + (long long)p1 * sp;
#pragma unroll
                for (int i = 0; i < EM; ++i) {
                    const int p = p1 + i * dp;
                    if (p < n) r[i] = cheb > 0 ? base[(long long)src(p) * sp] : q[i * step];
                }
#pragma unroll
                for (int i = 0; i < EM; ++i) {
                    const int p = p1 + i * dp;
                    if (p < n) dst[pidx(p)] = r[i];
                }
            }
        }
    }
    __syncthreads();
    const int col = tid >> a.wpc_log2;
    const bool act = col < TC;
    fft_lds<T, DIR>((act ? col : 0) * pitch, a.fft, reinterpret_cast<const cx<T> *>(a.tw),
                    act ? (tid & (wpc - 1)) : n, wpc);
    const int nout = cheb > 0 ? cheb : n;  // the DCT keeps outputs 0 .. cheb - 1
    {
        const bool out_rows = a.out_s.sc == 1;
        const int c = out_rows ? (tid & (TC - 1)) : (tid >> a.wpc_log2);
        const int p0 = out_rows ? (tid >> a.tc_log2) : (tid & (wpc - 1));
        const int dp = out_rows ? rows_per : wpc;
        const long long step = (long long)dp * a.out_s.sp;
        cx<T> *q = out + ob + (long long)c * a.out_s.sc + (long long)p0 * a.out_s.sp;
        const cx<T> *srcl = lds + c * pitch;
        if (c < ncol) {
            constexpr int EM = Stage<T>::value;
            for (int p1 = p0; p1 < nout; p1 += EM * dp, q += EM * step) {
                cx<T> r[EM];
#pragma unroll
                for (int i = 0; i < EM; ++i) r[i] = cmk<T>(T(0), T(0));
#pragma unroll
                for (int i = 0; i < EM; ++i) {
                    const int p = p1 + i * dp;
                    if (p < nout) r[i] = srcl[pidx(p)];
                }
#pragma unroll
                for (int i = 0; i < EM; ++i) {
                    const int p = p1 + i * dp;
                    if (p < nout) q[i * step] = r[i];
                }
            }
        }
    }
}

template <typename T, int DIR>
__global__ __launch_bounds__(kGenericThreads) void k_c2c_tile(PassArgs a) {
    c2c_tile_body<T, DIR>(a, a.in, a.out, blockIdx.x);
}

// Row offsets in the blocked workspace of the 2 TC real lines of an X tile:
// line g = z ny + y starts at row z zrows + y0 + y (column block 0).
__device__ __forceinline__ void x_row_offsets(const PassArgs &a, long long g0, int nl, long long *rowoff) {
    for (int l = threadIdx.x; l < nl; l += blockDim.x) {
        const long long g = g0 + l;
        const long long z = g / a.ny;
        const long long y = g - z * a.ny;
        rowoff[l] = (z * a.zrows + a.y0 + y) << a.b_log2;
    }
}

// ---- X stage, forward: real lines -> half spectra in the blocked workspace
template <typename T>
__device__ __forceinline__ void r2c_x_body(const PassArgs &a, const void *inp, void *outp, long long tile) {
    __shared__ long long rowoff[128];
    cx<T> *lds = reinterpret_cast<cx<T> *>(pf_smem);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int TC = 1 << a.tc_log2;
    const int wpc = 1 << a.wpc_log2;
    const int n = a.fft.n;
    const int pitch = a.pitch;
    const long long g0 = tile * (2 * TC);
    const T *__restrict__ in = reinterpret_cast<const T *>(inp);
    cx<T> *__restrict__ out = reinterpret_cast<cx<T> *>(outp);
    x_row_offsets(a, g0, 2 * TC, rowoff);
    const int c = tid >> a.wpc_log2;
    const bool act = c < TC;  // surplus threads of a batched launch only help with the stores
    if (act) {
        const long long ga = g0 + 2 * c, gb = ga + 1;
        const bool va = ga < a.lines, vb = gb < a.lines;
        const T *pa = in + ga * a.ld_real;
        const T *pb = in + gb * a.ld_real;
        // EM loads per line in flight before the first wait
        constexpr int EM = Stage<T>::value;
        for (int p1 = tid & (wpc - 1); p1 < n; p1 += EM * wpc) {
            T ra[EM], rb[EM];
#pragma unroll
            for (int i = 0; i < EM; ++i) {
                const int p = p1 + i * wpc;
                if (p < n) {
                    ra[i] = va ? pa[p] : T(0);
                    rb[i] = vb ? pb[p] : T(0);
                }
            }
#pragma unroll
            for (int i = 0; i < EM; ++i) {
                const int p = p1 + i * wpc;
                if (p < n) lds[c * pitch + pidx(p)] = cmk<T>(ra[i], rb[i]);
            }
        }
    }
    __syncthreads();
    fft_lds<T, -1>((act ? c : 0) * pitch, a.fft, reinterpret_cast<const cx<T> *>(a.tw),
                   act ? (tid & (wpc - 1)) : n, wpc);
    const int B = 1 << a.b_log2;
    const int total = a.nkb * TC * B;
    const long long kbstride = a.kbrows << a.b_log2;
    const T h = T(0.5);
    // modes f = (kb, cc, kk) of the tile, EH per thread at a time: LDS reads
    // first, then the split and the stores
    constexpr int EH = Stage<T>::value / 2;
    for (int f1 = tid; f1 < total; f1 += EH * nthr) {
        cx<T> zr[EH], wr[EH];
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int f = f1 + i * nthr;
            const int kk = f & (B - 1);
            const int cc = (f >> a.b_log2) & (TC - 1);
            const int k = (f >> (a.b_log2 + a.tc_log2)) * B + kk;
            if (f < total && k < a.nxh) {
                const cx<T> *col = lds + cc * pitch;
                zr[i] = col[pidx(k)];
                wr[i] = col[pidx(k == 0 ? 0 : n - k)];
            }
        }
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int f = f1 + i * nthr;
            const int kk = f & (B - 1);
            const int cc = (f >> a.b_log2) & (TC - 1);
            const int kb = f >> (a.b_log2 + a.tc_log2);
            const int k = kb * B + kk;
            const long long ga = g0 + 2 * cc;
            if (f < total && k < a.nxh && ga < a.lines) {
                const cx<T> z = zr[i], w = wr[i];
                out[rowoff[2 * cc] + kb * kbstride + kk] = cmk<T>((z.x + w.x) * h, (z.y - w.y) * h);
                if (ga + 1 < a.lines)
                    out[rowoff[2 * cc + 1] + kb * kbstride + kk] = cmk<T>((z.y + w.y) * h, (w.x - z.x) * h);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kGenericThreads) void k_r2c_x(PassArgs a) {
    r2c_x_body<T>(a, a.in, a.out, blockIdx.x);
}

// ---- X stage, backward: blocked half spectra -> real lines ---------------
template <typename T>
__device__ __forceinline__ void c2r_x_body(const PassArgs &a, const void *inp, void *outp, long long tile) {
    __shared__ long long rowoff[128];
    cx<T> *lds = reinterpret_cast<cx<T> *>(pf_smem);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int TC = 1 << a.tc_log2;
    const int wpc = 1 << a.wpc_log2;
    const int n = a.fft.n;
    const int pitch = a.pitch;
    const long long g0 = tile * (2 * TC);
    const cx<T> *__restrict__ in = reinterpret_cast<const cx<T> *>(inp);
    T *__restrict__ out = reinterpret_cast<T *>(outp);
    x_row_offsets(a, g0, 2 * TC, rowoff);
    __syncthreads();
    const int B = 1 << a.b_log2;
    const int total = a.nkb * TC * B;
    const long long kbstride = a.kbrows << a.b_log2;
    // modes f = (kb, cc, kk) of the tile, EH per thread at a time: all loads
    // in flight before the first wait, then the LDS writes
    constexpr int EH = Stage<T>::value / 2;
    for (int f1 = tid; f1 < total; f1 += EH * nthr) {
        cx<T> ra[EH], rb[EH];
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int f = f1 + i * nthr;
            const int kk = f & (B - 1);
            const int cc = (f >> a.b_log2) & (TC - 1);
            const int kb = f >> (a.b_log2 + a.tc_log2);
            const int k = kb * B + kk;
            const long long ga = g0 + 2 * cc;
            if (f < total && k < a.nxh && ga < a.lines) {
                ra[i] = in[rowoff[2 * cc] + kb * kbstride + kk];
                rb[i] = (ga + 1 < a.lines) ? in[rowoff[2 * cc + 1] + kb * kbstride + kk] : cmk<T>(T(0), T(0));
            }
        }
#pragma unroll
        for (int i = 0; i < EH; ++i) {
            const int f = f1 + i * nthr;
            const int kk = f & (B - 1);
            const int cc = (f >> a.b_log2) & (TC - 1);
            const int k = (f >> (a.b_log2 + a.tc_log2)) * B + kk;
            const long long ga = g0 + 2 * cc;
            if (f < total && k < a.nxh && ga < a.lines) {
                const cx<T> xa = ra[i], xb = rb[i];
                cx<T> *col = lds + cc * pitch;
                if (k == 0 || 2 * k == n) {
                    col[pidx(k)] = cmk<T>(xa.x, xb.x);
                } else {
                    col[pidx(k)] = cmk<T>(xa.x - xb.y, xa.y + xb.x);
                    col[pidx(n - k)] = cmk<T>(xa.x + xb.y, xb.x - xa.y);
                }
            }
        }
    }
    __syncthreads();
    const int c = tid >> a.wpc_log2;
    const bool act = c < TC;
    fft_lds<T, 1>((act ? c : 0) * pitch, a.fft, reinterpret_cast<const cx<T> *>(a.tw),
                  act ? (tid & (wpc - 1)) : n, wpc);
    if (act) {
        const long long ga = g0 + 2 * c, gb = ga + 1;
        const bool va = ga < a.lines, vb = gb < a.lines;
        T *pa = out + ga * a.ld_real;
        T *pb = out + gb * a.ld_real;
        const cx<T> *col = lds + c * pitch;
        constexpr int EM = Stage<T>::value;
        for (int p1 = tid & (wpc - 1); p1 < n; p1 += EM * wpc) {
            cx<T> r[EM];
#pragma unroll
            for (int i = 0; i < EM; ++i) {
                const int p = p1 + i * wpc;
                if (p < n) r[i] = col[pidx(p)];
            }
#pragma unroll
            for (int i = 0; i < EM; ++i) {
                const int p = p1 + i * wpc;
                if (p < n) {
                    if (va) pa[p] = r[i].x;
                    if (vb) pb[p] = r[i].y;
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kGenericThreads) void k_c2r_x(PassArgs a) {
    c2r_x_body<T>(a, a.in, a.out, blockIdx.x);
}

// ---- batched passes: one launch over the tiles of many transforms --------
// Block b belongs to the transform i with first[i] <= b < first[i + 1] (a
// binary search over the table, uniform per block) and works on its tile
// b - first[i] with that transform's arguments args[i].  A pointer of
// args[i] that names a user array holds a byte offset from the call's base.
__device__ __forceinline__ int batch_find(const BatchArgs &b, long long blk) {
    int lo = 0, hi = b.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.first[mid] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ const void *batch_in(const BatchArgs &b, const PassArgs &a) {
    return b.in_user ? (const void *)(b.user_in + (size_t)a.in) : a.in;
}
__device__ __forceinline__ void *batch_out(const BatchArgs &b, const PassArgs &a) {
    return b.out_user ? (void *)(b.user_out + (size_t)a.out) : a.out;
}

template <typename T, int DIR>
__global__ __launch_bounds__(kGenericThreads) void k_c2c_tile_b(BatchArgs b) {
    const long long blk = blockIdx.x;
    const int i = batch_find(b, blk);
    const PassArgs &a = b.args[i];
    c2c_tile_body<T, DIR>(a, batch_in(b, a), batch_out(b, a), blk - b.first[i]);
}

template <typename T>
__global__ __launch_bounds__(kGenericThreads) void k_r2c_x_b(BatchArgs b) {
    const long long blk = blockIdx.x;
    const int i = batch_find(b, blk);
    const PassArgs &a = b.args[i];
    r2c_x_body<T>(a, batch_in(b, a), batch_out(b, a), blk - b.first[i]);
}

template <typename T>
__global__ __launch_bounds__(kGenericThreads) void k_c2r_x_b(BatchArgs b) {
    const long long blk = blockIdx.x;
    const int i = batch_find(b, blk);
    const PassArgs &a = b.args[i];
    c2r_x_body<T>(a, batch_in(b, a), batch_out(b, a), blk - b.first[i]);
}

hipError_t launch_batch(const BatchLaunch &L, hipStream_t s) {
    if (L.blocks == 0) return hipSuccess;
    if (L.kind == PASS_C2C_MR || L.kind == PASS_R2C_MR || L.kind == PASS_C2R_MR) return mr_launch_batch(L, s);
    if (L.threads == 0 || L.threads > (unsigned)kGenericThreads) return hipErrorInvalidConfiguration;
    const dim3 g(L.blocks), bl(L.threads);
    const bool f64 = L.prec != 0;
    switch (L.kind) {
        case PASS_C2C:
            if (f64) {
                if (L.dir < 0) hipLaunchKernelGGL((k_c2c_tile_b<double, -1>), g, bl, L.lds, s, L.b);
                else hipLaunchKernelGGL((k_c2c_tile_b<double, 1>), g, bl, L.lds, s, L.b);
            } else {
                if (L.dir < 0) hipLaunchKernelGGL((k_c2c_tile_b<float, -1>), g, bl, L.lds, s, L.b);
                else hipLaunchKernelGGL((k_c2c_tile_b<float, 1>), g, bl, L.lds, s, L.b);
            }
            break;
        case PASS_R2C_X:
            if (f64) hipLaunchKernelGGL(k_r2c_x_b<double>, g, bl, L.lds, s, L.b);
            else hipLaunchKernelGGL(k_r2c_x_b<float>, g, bl, L.lds, s, L.b);
            break;
        case PASS_C2R_X:
            if (f64) hipLaunchKernelGGL(k_c2r_x_b<double>, g, bl, L.lds, s, L.b);
            else hipLaunchKernelGGL(k_c2r_x_b<float>, g, bl, L.lds, s, L.b);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---- pack / unpack between the global arrays and the Table 1 blocks ------
// An axis of length n split over M ranks: rank r holds floor(n/M) + (r < n mod M)
// elements starting at r floor(n/M) + min(r, n mod M) (blocks differ by at most
// one element, Sec. 3.4).
__device__ __forceinline__ void blk(int n, int M, int r, int &start, int &size) {
    const int q = n / M, rem = n % M;
    size = q + (r < rem ? 1 : 0);
    start = r * q + (r < rem ? r : rem);
}
__device__ __forceinline__ int block_of(int i, int n, int M) {
    const int q = n / M, rem = n % M;
    return i < rem * (q + 1) ? i / (q + 1) : rem + (i - rem * (q + 1)) / q;
}

// One line per workgroup; the block of rank (r1, r2) starts where the blocks
// of all earlier ranks (order r2 m1 + r1) end, which in closed form is
// nx (ny z0 + y0 L3) for X-pencils and nz (nxh ky0 + kx0 Ly) for Z-pencils.
__global__ __launch_bounds__(256) void k_remap(RemapArgs a) {
    const long long L = blockIdx.x;
    long long goff, boff;
    int len;
    if (a.kind == REMAP_XPENCIL) {
        const int z = (int)(L / a.ny), y = (int)(L - (long long)z * a.ny);
        int y0, L2, z0, L3;
        blk(a.ny, a.m1, block_of(y, a.ny, a.m1), y0, L2);
        blk(a.nz, a.m2, block_of(z, a.nz, a.m2), z0, L3);
        len = a.nx;
        goff = L * a.nx;
        boff = (long long)a.nx * ((long long)a.ny * z0 + (long long)y0 * L3 + (long long)(z - z0) * L2 + (y - y0));
    } else if (a.kind == REMAP_ZSTRIDE1) {
        const int kx = (int)(L / a.ny), ky = (int)(L - (long long)kx * a.ny);
        int kx0, Lx, ky0, Ly;
        blk(a.nxh, a.m1, block_of(kx, a.nxh, a.m1), kx0, Lx);
        blk(a.ny, a.m2, block_of(ky, a.ny, a.m2), ky0, Ly);
        len = a.nz;
        goff = L * a.nz;
        boff = (long long)a.nz *
               ((long long)a.nxh * ky0 + (long long)kx0 * Ly + (long long)(kx - kx0) * Ly + (ky - ky0));
    } else {
        const int r1 = (int)(L % a.m1);
        const long long row = L / a.m1;  // kz ny + ky
        const int kz = (int)(row / a.ny), ky = (int)(row - (long long)kz * a.ny);
        int kx0, Lx, ky0, Ly;
        blk(a.nxh, a.m1, r1, kx0, Lx);
        blk(a.ny, a.m2, block_of(ky, a.ny, a.m2), ky0, Ly);
        len = Lx;
        goff = row * a.nxh + kx0;
        boff = (long long)a.nz * ((long long)a.nxh * ky0 + (long long)kx0 * Ly) +
               ((long long)kz * Ly + (ky - ky0)) * Lx;
    }
    const unsigned *__restrict__ src = reinterpret_cast<const unsigned *>(a.src);
    unsigned *__restrict__ dst = reinterpret_cast<unsigned *>(a.dst);
    const long long so = (a.gather ? boff : goff) * a.words;
    const long long d0 = (a.gather ? goff : boff) * a.words;
    const int nw = len * a.words;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[d0 + i] = src[so + i];
}

// Zero the workspace elements of the boxes of f: one thread per 16-byte chunk
// of a 128-byte row (grid-stride), per-element stores where a chunk meets the
// kept mode range.
__global__ __launch_bounds__(256) void k_fill(FillArgs f) {
    float4 *__restrict__ w = reinterpret_cast<float4 *>(f.w);
    float *__restrict__ wf = reinterpret_cast<float *>(f.w);
    constexpr int CH = 8;          // 16-byte chunks per row
    const int epc = 4 / f.words;   // elements per chunk (2 FP32 complex, 1 FP64 complex)
    for (int b = 0; b < f.nbox; ++b) {
        const int nz = f.z1[b] - f.z0[b], nk = f.kb1[b] - f.kb0[b], ny = f.y1[b] - f.y0[b];
        if (nz <= 0 || nk <= 0 || ny <= 0) continue;
        const long long total = (long long)nz * nk * ny * CH;
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
             i += (long long)gridDim.x * blockDim.x) {
            const int c = (int)(i & (CH - 1));
            long long r = i >> 3;
            const int y = (int)(r % ny);
            r /= ny;
            const int kb = f.kb0[b] + (int)(r % nk);
            const int z = f.z0[b] + (int)(r / nk);
            const long long row = (long long)z * f.zrows + (long long)kb * f.kbrows + f.y0[b] + y;
            const int kx0 = kb * f.B + c * epc;  // first mode of the chunk
            const long long at = row * CH + c;
            if (kx0 + epc <= f.keep0 || kx0 >= f.keep1) {
                w[at] = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                for (int e = 0; e < epc; ++e)
                    if (kx0 + e < f.keep0 || kx0 + e >= f.keep1)
                        for (int q = 0; q < f.words; ++q) wf[at * 4 + e * f.words + q] = 0.f;
            }
        }
    }
}

// One block per box row (i1, i2); threads copy the row's s0 elements.
__global__ __launch_bounds__(256) void k_box(BoxArgs b) {
    const int i1 = (int)(blockIdx.x % b.s1), i2 = (int)(blockIdx.x / b.s1);
    const long long g = ((long long)(b.o2 + i2) * b.st2 + (long long)(b.o1 + i1) * b.st1 + b.o0) * b.words;
    const long long k = ((long long)i2 * b.s1 + i1) * b.s0 * b.words;
    const unsigned *__restrict__ src = reinterpret_cast<const unsigned *>(b.src);
    unsigned *__restrict__ dst = reinterpret_cast<unsigned *>(b.dst);
    const long long so = b.to_block ? g : k, d0 = b.to_block ? k : g;
    const int nw = b.s0 * b.words;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[d0 + i] = src[so + i];
}

hipError_t launch_fill(const FillArgs &f, hipStream_t s) {
    if (f.nbox < 0 || f.nbox > 4 || f.B * f.words != 32) return hipErrorInvalidValue;
    long long total = 0;
    for (int b = 0; b < f.nbox; ++b) {
        const long long nz = f.z1[b] - f.z0[b], nk = f.kb1[b] - f.kb0[b], ny = f.y1[b] - f.y0[b];
        if (nz > 0 && nk > 0 && ny > 0) total = std::max(total, nz * nk * ny * 8);
    }
    if (total <= 0) return hipSuccess;
    const long long want = (total + 255) / 256;
    const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_box(const BoxArgs &b, hipStream_t s) {
    const long long rows = (long long)b.s1 * b.s2;
    if (rows <= 0 || b.s0 <= 0) return hipSuccess;
    if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_box, dim3((unsigned)rows), dim3(256), 0, s, b);
    return hipGetLastError();
}

// ---- spectral step: the diagonal multiplier and the DCT end-node weights ---
template <typename T>
__global__ __launch_bounds__(256) void k_spec_mul(SpecArgs a) {
    const long long total = (long long)a.nxh * a.ny * a.nz;
    cx<T> *U = reinterpret_cast<cx<T> *>(a.U);
    const double two_pi = 6.283185307179586476925286766559;
    const double pi = 3.1415926535897932384626433832795;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int kx, ky, kz;
        if (a.stride1) {  // [kx][ky][kz]
            kz = (int)(e % a.nz);
            const long long r = e / a.nz;
            ky = (int)(r % a.ny);
            kx = (int)(r / a.ny);
        } else {  // [kz][ky][kx]
            kx = (int)(e % a.nxh);
            const long long r = e / a.nxh;
            ky = (int)(r % a.ny);
            kz = (int)(r / a.ny);
        }
        const int kys = 2 * ky <= a.ny ? ky : ky - a.ny;
        const double kxr = two_pi * kx / a.nx, kyr = two_pi * kys / a.ny, kzr = pi * kz / (a.nz - 1);
        const double k2 = kxr * kxr + kyr * kyr + kzr * kzr;
        const double mu = k2 > 0.0 ? -a.scale * kxr / k2 : 0.0;  // m = i mu
        const double sg = a.conj ? -1.0 : 1.0;
        const cx<T> u = U[e];
        // u * (i sg mu) = (-sg mu u.y, sg mu u.x)
        U[e] = cmk<T>((T)(-sg * mu * (double)u.y), (T)(sg * mu * (double)u.x));
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zweight(const T *__restrict__ src, T *__restrict__ dst, int plane, int nz,
                                                 int e) {
    const long long total = (long long)plane * nz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(i / plane);
        const T w = (z == 0 || z == nz - 1) ? T(1) : (e > 0 ? T(2) : T(0.5));
        dst[i] = src[i] * w;
    }
}

static unsigned grid_for(long long total) {
    const long long b = (total + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

hipError_t launch_spec_mul(const SpecArgs &a, hipStream_t s) {
    const long long total = (long long)a.nxh * a.ny * a.nz;
    if (a.f64) hipLaunchKernelGGL(k_spec_mul<double>, dim3(grid_for(total)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_spec_mul<float>, dim3(grid_for(total)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zweight(const void *src, void *dst, int nx, int ny, int nz, int f64, int e, hipStream_t s) {
    const int plane = nx * ny;
    const long long total = (long long)plane * nz;
    if (f64)
        hipLaunchKernelGGL(k_zweight<double>, dim3(grid_for(total)), dim3(256), 0, s,
                           reinterpret_cast<const double *>(src), reinterpret_cast<double *>(dst), plane, nz, e);
    else
        hipLaunchKernelGGL(k_zweight<float>, dim3(grid_for(total)), dim3(256), 0, s,
                           reinterpret_cast<const float *>(src), reinterpret_cast<float *>(dst), plane, nz, e);
    return hipGetLastError();
}

hipError_t launch_remap(const RemapArgs &r, hipStream_t s) {
    if (r.nlines <= 0) return hipSuccess;
    if (r.nlines > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_remap, dim3((unsigned)r.nlines), dim3(256), 0, s, r);
    return hipGetLastError();
}

// Plain HBM copy, 16 bytes per lane, a fixed number of 16-byte words per
// thread (all loads issued before the stores).  The bandwidth this reaches is
// the practical ceiling the transform passes are measured against.
__global__ __launch_bounds__(512) void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n) {
    constexpr int U = 4;
    const size_t base = (size_t)blockIdx.x * blockDim.x * U + threadIdx.x;
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * blockDim.x;
        if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t i = base + (size_t)u * blockDim.x;
        if (i < n) dst[i] = v[u];
    }
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const size_t per_block = 512 * 4;
    const size_t blocks = (n + per_block - 1) / per_block;
    if (blocks > 0x7fffffffULL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(512), 0, s, reinterpret_cast<const float4 *>(src),
                       reinterpret_cast<float4 *>(dst), n);
    return hipGetLastError();
}

// The transform passes' access shape without the transform: persistent
// workgroups (one per CU) of 1024 threads move 128 KB tiles (8 loads of 16
// bytes per thread), tile t, t + gridDim.x, ...; the next tile's loads are in
// flight while the current one is stored; nontemporal loads and stores.
// src == dst reads and writes back each tile in place (the Y pass's pattern).
// Of the shapes measured (256 .. 1024 threads, 4 .. 32 loads per thread, with
// and without prefetch or hints, 1 .. 8 workgroups per CU) this one was the
// fastest.
__global__ __launch_bounds__(1024) void k_copy_tiles(const float4 *src, float4 *dst, size_t n) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    constexpr int U = 8, TPB = 1024;
    const size_t tile = (size_t)TPB * U;  // 16-byte words per tile
    const size_t ntiles = (n + tile - 1) / tile;
    const f4v *s = reinterpret_cast<const f4v *>(src);
    f4v *d = reinterpret_cast<f4v *>(dst);
    f4v cur[U], nxt[U];
    auto load = [&](f4v(&v)[U], size_t t) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = t * tile + (size_t)u * TPB + threadIdx.x;
            if (i < n) v[u] = __builtin_nontemporal_load(s + i);
        }
    };
    size_t t = blockIdx.x;
    if (t < ntiles) load(nxt, t);
    for (; t < ntiles; t += gridDim.x) {
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
        if (t + gridDim.x < ntiles) load(nxt, t + gridDim.x);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t i = t * tile + (size_t)u * TPB + threadIdx.x;
            if (i < n) __builtin_nontemporal_store(cur[u], d + i);
        }
    }
}

hipError_t launch_copy_tiles(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    int dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t tiles = (n + 1024 * 8 - 1) / (1024 * 8);
    const unsigned blocks = (unsigned)(tiles < (size_t)ncu ? tiles : (size_t)ncu);
    hipLaunchKernelGGL(k_copy_tiles, dim3(blocks), dim3(1024), 0, s, reinterpret_cast<const float4 *>(src),
                       reinterpret_cast<float4 *>(dst), n);
    return hipGetLastError();
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t prepare_kernels(size_t max_lds) {
    hipError_t e = hipSuccess;
#define PF_ALLOW(k)                                      \
    do {                                                 \
        hipError_t r = allow_lds(k, max_lds);            \
        if (r != hipSuccess && e == hipSuccess) e = r;   \
    } while (0)
    PF_ALLOW((k_c2c_tile<float, -1>));
    PF_ALLOW((k_c2c_tile<float, 1>));
    PF_ALLOW((k_c2c_tile<double, -1>));
    PF_ALLOW((k_c2c_tile<double, 1>));
    PF_ALLOW(k_r2c_x<float>);
    PF_ALLOW(k_r2c_x<double>);
    PF_ALLOW(k_c2r_x<float>);
    PF_ALLOW(k_c2r_x<double>);
    PF_ALLOW((k_c2c_tile_b<float, -1>));
    PF_ALLOW((k_c2c_tile_b<float, 1>));
    PF_ALLOW((k_c2c_tile_b<double, -1>));
    PF_ALLOW((k_c2c_tile_b<double, 1>));
    PF_ALLOW(k_r2c_x_b<float>);
    PF_ALLOW(k_r2c_x_b<double>);
    PF_ALLOW(k_c2r_x_b<float>);
    PF_ALLOW(k_c2r_x_b<double>);
#undef PF_ALLOW
    return e;
}

hipError_t launch_pass(const PassDesc &d, hipStream_t s) {
    const dim3 g(d.blocks), b(d.threads);
    const bool f64 = d.prec != 0;
    const bool generic = d.kind == PASS_C2C || d.kind == PASS_R2C_X || d.kind == PASS_C2R_X;
    if (generic && (d.threads == 0 || d.threads > (unsigned)kGenericThreads)) return hipErrorInvalidConfiguration;
    switch (d.kind) {
        case PASS_C2C:
            if (f64) {
                if (d.dir < 0)
                    hipLaunchKernelGGL((k_c2c_tile<double, -1>), g, b, d.lds, s, d.a);
                else
                    hipLaunchKernelGGL((k_c2c_tile<double, 1>), g, b, d.lds, s, d.a);
            } else {
                if (d.dir < 0)
                    hipLaunchKernelGGL((k_c2c_tile<float, -1>), g, b, d.lds, s, d.a);
                else
                    hipLaunchKernelGGL((k_c2c_tile<float, 1>), g, b, d.lds, s, d.a);
            }
            break;
        case PASS_R2C_X:
            if (f64)
                hipLaunchKernelGGL(k_r2c_x<double>, g, b, d.lds, s, d.a);
            else
                hipLaunchKernelGGL(k_r2c_x<float>, g, b, d.lds, s, d.a);
            break;
        case PASS_C2R_X:
            if (f64)
                hipLaunchKernelGGL(k_c2r_x<double>, g, b, d.lds, s, d.a);
            else
                hipLaunchKernelGGL(k_c2r_x<float>, g, b, d.lds, s, d.a);
            break;
        case PASS_C2C_P2:
        case PASS_R2C_P2:
        case PASS_C2R_P2:
            return p2_launch(d, s);
        case PASS_REMAP:
            return launch_remap(d.r, s);
        case PASS_FILL:
            return launch_fill(d.f, s);
        case PASS_BOX:
            return launch_box(d.b, s);
        case PASS_C2C_MR:
        case PASS_R2C_MR:
        case PASS_C2R_MR:
            return mr_launch(d, s);
        case PASS_FUSED_XY:  // launched by the planner (p2_fused_launch), which holds its arguments
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pf
