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
#include "fft_device.h"
#include "pf_internal.h"

namespace pf {

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
// The row xor and the pair xor keep every exchange pattern of the kernel
// free of bank conflicts for N = 512 and 1024 (64 banks of 4 bytes).
template <int TC>
__device__ __forceinline__ int p2_slot(int p, int cp) {
    constexpr int CP = TC / 2;
    return ((p ^ ((p >> 4) & 1)) * CP) + (cp ^ (((p >> 1) ^ (p >> 5)) & (CP - 1)));
}

// One stage's butterflies on the 16 registers of a column: butterfly i
// (j = q + i N/16) takes v[i + r 16/R], r < R, twiddles by W_{NS R}^{r k},
// k = j mod NS, and leaves its R outputs in the same registers.
template <int N, int R, int NS, int DIR>
__device__ __forceinline__ void p2_butterflies(cx<float> (&v)[16], int q, const cx<float> *tws) {
    constexpr int T = N / 16;
    constexpr int BPT = 16 / R;
#pragma unroll
    for (int i = 0; i < BPT; ++i) {
        const int j = q + i * T;
        const int k = j & (NS - 1);
        cx<float> w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = v[i + r * BPT];
        if (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<float> t = tws[k * (R - 1) + r - 1];
                if (DIR > 0) t.y = -t.y;
                w[r] = cmul(w[r], t);
            }
        }
        Dft<float, R, DIR>::run(w);
#pragma unroll
        for (int r = 0; r < R; ++r) v[i + r * BPT] = w[r];
    }
}

__device__ __forceinline__ float4 pack2(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }

// Each thread owns a pair of adjacent columns (2 cp, 2 cp + 1) and 16 points
// q + (N/16) m of both.  INP / OUTP: 1 if that side's points are contiguous
// (lines), 0 if its columns are contiguous (rows, loaded 16 bytes at a time).
template <int N, int TC, int DIR, int INP, int OUTP>
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

    const cx<float> *__restrict__ in = reinterpret_cast<const cx<float> *>(a.in);
    cx<float> *__restrict__ out = reinterpret_cast<cx<float> *>(a.out);
    const int CB = (int)a.CB;
    const int ntiles = (int)(a.A * a.CB);
    const int cp_in = INP ? tid / T : tid % CP;
    const int q_in = INP ? tid % T : tid / CP;
    const int cp_mid = tid % CP;
    const int q_mid = tid / CP;
    const int cp_out = OUTP ? tid / T : tid % CP;
    const int q_out = OUTP ? tid % T : tid / CP;
    const long long in_step = a.in_s.sp * T;
    const long long out_step = a.out_s.sp * T;

    // element (column 2 cp, point q) of tile t on a side, and the valid column count
    auto side_addr = [&](const Side &sd, int t, int cp, int q, int &ncol) -> long long {
        const int ta = t / CB;
        const int cb = t - ta * CB;
        ncol = min(TC, a.C - cb * TC);
        return (long long)ta * sd.sa + (long long)(cb / sd.cpb) * sd.sblk + (long long)(cb % sd.cpb) * TC * sd.sc +
               (long long)(2 * cp) * sd.sc + (long long)q * sd.sp;
    };
    auto load = [&](cx<float>(&d0)[16], cx<float>(&d1)[16], int t) {
        int ncol;
        const long long b = side_addr(a.in_s, t, cp_in, q_in, ncol);
        if (INP) {  // two lines, 8 bytes per lane each
            if (2 * cp_in < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m) d0[m] = in[b + m * in_step];
            }
            if (2 * cp_in + 1 < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m) d1[m] = in[b + a.in_s.sc + m * in_step];
            }
        } else if (2 * cp_in < ncol) {  // rows: both columns in one 16-byte load
            // a partially valid pair only occurs on a side padded to whole 16-column blocks
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = *reinterpret_cast<const float4 *>(in + b + m * in_step);
                d0[m] = make_float2(x.x, x.y);
                d1[m] = make_float2(x.z, x.w);
            }
        }
    };

    int t = blockIdx.x;
    cx<float> p0[16], p1[16];
    if (t < ntiles) load(p0, p1, t);
    __syncthreads();  // twiddle table in LDS
    for (; t < ntiles; t += gridDim.x) {
        cx<float> v0[16], v1[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            v0[m] = p0[m];
            v1[m] = p1[m];
        }
        const int tn = t + gridDim.x;
        if (tn < ntiles) load(p0, p1, tn);

        // stage 0: radix 16 on x[q + T r], outputs to points 16 q + r
        Dft<float, 16, DIR>::run(v0);
        Dft<float, 16, DIR>::run(v1);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[p2_slot<TC>(q_in * 16 + r, cp_in)] = pack2(v0[r], v1[r]);
        __syncthreads();

        if constexpr (S == 3) {  // stage 1: radix 16, NS = 16
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const float4 x = buf[p2_slot<TC>(q_mid + T * m, cp_mid)];
                v0[m] = make_float2(x.x, x.y);
                v1[m] = make_float2(x.z, x.w);
            }
            __syncthreads();
            p2_butterflies<N, 16, 16, DIR>(v0, q_mid, twl + p2_twoff(N, 1));
            p2_butterflies<N, 16, 16, DIR>(v1, q_mid, twl + p2_twoff(N, 1));
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
        p2_butterflies<N, RL, NSL, DIR>(v0, q_out, twl + p2_twoff(N, S - 1));
        p2_butterflies<N, RL, NSL, DIR>(v1, q_out, twl + p2_twoff(N, S - 1));
        {
            int ncol;
            const long long b = side_addr(a.out_s, t, cp_out, q_out, ncol);
            if (OUTP) {
                if (2 * cp_out < ncol) {
#pragma unroll
                    for (int m = 0; m < 16; ++m) out[b + m * out_step] = v0[m];
                }
                if (2 * cp_out + 1 < ncol) {
#pragma unroll
                    for (int m = 0; m < 16; ++m) out[b + a.out_s.sc + m * out_step] = v1[m];
                }
            } else if (2 * cp_out < ncol) {
#pragma unroll
                for (int m = 0; m < 16; ++m)
                    *reinterpret_cast<float4 *>(out + b + m * out_step) = pack2(v0[m], v1[m]);
            }
        }
        __syncthreads();  // the next tile's stage 0 overwrites the LDS tile
    }
}

int p2_tc(int n) { return n <= 1024 ? 16 : 16384 / n; }

size_t p2_lds_bytes(int n) { return ((size_t)n * p2_tc(n) + n) * sizeof(float2); }

bool p2_supported(int n, int prec) {
    return prec == 0 && (n == 256 || n == 512 || n == 1024 || n == 2048 || n == 4096);
}

template <int N, int TC, int DIR, int INP, int OUTP>
static const void *p2_kernel() {
    return reinterpret_cast<const void *>(&k_c2c_p2<N, TC, DIR, INP, OUTP>);
}

// kernel symbol for (n, dir, inp, outp); nullptr if not built
static const void *p2_pick(int n, int dir, int inp, int outp) {
#define PF_P2_DIRS(NV, TCV)                                                   \
    if (n == NV) {                                                            \
        if (dir < 0) {                                                        \
            if (!inp && !outp) return p2_kernel<NV, TCV, -1, 0, 0>();         \
            if (!inp && outp) return p2_kernel<NV, TCV, -1, 0, 1>();          \
            if (inp && !outp) return p2_kernel<NV, TCV, -1, 1, 0>();          \
        } else {                                                              \
            if (!inp && !outp) return p2_kernel<NV, TCV, 1, 0, 0>();          \
            if (!inp && outp) return p2_kernel<NV, TCV, 1, 0, 1>();           \
            if (inp && !outp) return p2_kernel<NV, TCV, 1, 1, 0>();           \
        }                                                                     \
        return nullptr;                                                       \
    }
    PF_P2_DIRS(256, 16)
    PF_P2_DIRS(512, 16)
    PF_P2_DIRS(1024, 16)
    PF_P2_DIRS(2048, 8)
    PF_P2_DIRS(4096, 4)
#undef PF_P2_DIRS
    return nullptr;
}

const void *p2_symbol(const PassDesc &d) { return p2_pick(d.a.fft.n, d.dir, d.a.inp, d.a.outp); }

hipError_t p2_prepare(int n) {
    const size_t lds = p2_lds_bytes(n);
    hipError_t e = hipSuccess;
    for (int dir : {-1, 1})
        for (int io = 0; io < 3; ++io) {
            const void *k = p2_pick(n, dir, io == 2, io == 1);
            if (!k) continue;
            hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
