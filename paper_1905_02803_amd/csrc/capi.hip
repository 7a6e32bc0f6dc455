// capi.hip -- host side of the pencil 3D FFT library: validation, Table 1
// layout arithmetic, radix plans, twiddle tables, workspace and the pass
// chain behind the C ABI of include/pencilfft.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pencilfft.h"
#include "pf_internal.h"

using pf::FftSpec;
using pf::PassArgs;
using pf::PassDesc;
using pf::Side;

namespace {

constexpr int kPasses = 6;  // at most: fill, insert, Z, Y, mask, X (share-only backward)
constexpr size_t kLdsBudget = 80 * 1024;  // two workgroups per CU fit in 160 KB

struct EventPair {
    hipEvent_t start, stop;
};

struct PassTiming {
    std::vector<EventPair> used;
};

// Plan choices beyond the layout: the batched transforms use the generic
// kernels only (one kernel kind per pass type across the batch), take their
// workspace from the batch, and may carry tuned radix orders and tile widths
// per axis (x, y, z): radix_order 0 = 16, 8, 4, 2, 3, 5, 7; 1 = 8, 4, 2, 3, 5,
// 7; 2 = 4, 2, 3, 5, 7; 3 = 3, 5, 7, 16, 8, 4, 2; tile 0 = the default widest
// tile, else at most `tile` line pairs (x) or columns (y, z) per tile.
struct PlanOpts {
    bool generic_only = false;
    bool no_mr = false;  // keep the runtime-radix kernels where a compile-time mixed-radix one exists
    bool no_spec_sr = false;  // fused spectral step by the even extension even where the split form exists
    bool no_bwd_tr = false;  // backward chain on W (no transposed workspace)
    bool no_fwd_tr = false;  // forward chain on W (no transposed workspace)
    bool external_ws = false;
    int radix_order[3] = {0, 0, 0};
    int tile[3] = {0, 0, 0};
};

}  // namespace

struct pf_plan {
    int nx, ny, nz, nxh;
    int ncu;  // compute units of the device the plan was made on
    pf_layout lay;
    int csize;  // bytes per complex value
    int B, b_log2, nkb;
    long long zrows, kbrows;  // W rows (of B modes) between z planes / column blocks
    FftSpec fx, fy, fz;
    void *tw_dev;  // one allocation holding the x, y, z tables (+ the half-length X table)
    size_t tw_off[4];
    // x, y, z: a compile-time mixed-radix kernel serves the axis (FP32), and the
    // offset of its table W_n^m, m < n, in tw_dev
    bool mr[3];
    size_t tw_mr[3];
    size_t tw_dct;  // split type-I DCT of the fused spectral step: [L-point][M-point stage tables][W_4M^k]
    bool spec_sr;
    FftSpec fxh;   // nx / 2 plan of the even power-of-two X stage
    bool fast_x;
    void *ws;          // the workspace: W, then (m1 m2 > 1) the global-array buffer
    size_t ws_bytes;
    size_t w_bytes;    // bytes of W
    // backward chain on the transposed workspace W' = complex [nz][nxh][ny]
    // (rows of 16 ky lines at one kx): the Z pass reads 16 adjacent Z-pencil
    // lines per tile, the Y pass runs in place along the contiguous ky lines, the
    // X pass reads rows of 16 lines at one mode.  FP32 plain, STRIDE1 1 x 1
    // plans with a power-of-two X pass and ny a multiple of 16 up to 512; W'
    // fits in W.  Measured per pair: 512^3 1.37 -> 1.35 ms, 1024 x 512 x 1024
    // 5.21 -> 5.09 ms, 2048 x 512 x 512 5.57 -> 5.29 ms; at ny = 1024 (1024^3,
    // 9.83 -> 10.0 ms) the Y pass along 8 KB lines and the X pass's rows 8 KB
    // apart lose more than the Z pass gains, so W stays there.
    bool bwd_tr, fwd_tr;
    bool own_ws;
    bool blocked;      // m1 m2 > 1: user arrays are the concatenated Table 1 blocks
    bool share;        // share-only: user arrays are rank (r1, r2)'s blocks
    size_t so_x, so_y, so_zw, so_zg;  // share-only byte offsets: X and Y into W, Z into W and G
    int npass[2];
    PassDesc pass[2][kPasses];
    const char *pass_names[2][kPasses];
    double pass_bytes[2][kPasses];
    // Chebyshev third transform with a power-of-two extension (FP32, 1 x 1):
    // the spectral step's Z passes and product fused into one pass on W
    bool spec_fused;
    PassDesc spec;
    // fused X-Y passes (pf_layout.fused_xy): their arguments per direction
    // and the device counters they share (queue tickets, plane counts, status)
    bool fused;
    pf::FusedArgs fxy[2];
    unsigned fused_blocks;
    int fused_nq;  // work queues: the XCDs the fused launch's workgroups run on
    unsigned *ctl;
    bool timing;
    PassTiming tim[2][kPasses];
    std::vector<EventPair> pool;
    PlanOpts opt;
};

namespace {

int ilog2(long long v) {
    int r = 0;
    while ((1LL << r) < v) ++r;
    return r;
}

bool valid_layout_values(const pf_layout *l) {
    if (l->m1 < 1 || l->m2 < 1) return false;
    if (l->stride1 != 0 && l->stride1 != 1) return false;
    if (l->useeven != 0 && l->useeven != 1) return false;
    if (l->precision != PF_F32 && l->precision != PF_F64) return false;
    if (l->math != PF_PLAIN && l->math != PF_MFMA_FP16X2 && l->math != PF_MFMA_BF16X2) return false;
    if (l->inplace != 0 && l->inplace != 1) return false;
    if (l->third != PF_THIRD_FFT && l->third != PF_THIRD_EMPTY && l->third != PF_THIRD_CHEB) return false;
    if (l->share_only != 0 && l->share_only != 1) return false;
    if (l->fused_xy != 0 && l->fused_xy != 1) return false;
    if (l->share_only) {
        if (l->r1 < 0 || l->r1 >= l->m1 || l->r2 < 0 || l->r2 >= l->m2) return false;
    } else if (l->r1 != 0 || l->r2 != 0) {
        return false;
    }
    return true;
}

// Radix plan: by default 16s first, then 8, 4, 2, then 3, 5, 7 (PlanOpts
// lists the other orders); returns false for other primes.
bool factor_length(int n, FftSpec *fs, int order_code = 0) {
    std::memset(fs, 0, sizeof(*fs));
    fs->n = n;
    int m = n, s = 0;
    static const int orders[4][7] = {{16, 8, 4, 2, 3, 5, 7}, {8, 4, 2, 3, 5, 7, 0}, {4, 2, 3, 5, 7, 0, 0},
                                     {3, 5, 7, 16, 8, 4, 2}};
    const int *order = orders[order_code >= 0 && order_code < 4 ? order_code : 0];
    for (int oi = 0; oi < 7; ++oi) {
        const int r = order[oi];
        if (r == 0) break;
        while (m % r == 0 && m > 1) {
            if (s >= pf::kMaxStages) return false;
            fs->radix[s++] = r;
            m /= r;
        }
    }
    if (m != 1) return false;
    fs->nstages = s;
    int off = 0, Ns = 1;
    for (int i = 0; i < s; ++i) {
        fs->twoff[i] = off;
        off += Ns * (fs->radix[i] - 1);
        Ns *= fs->radix[i];
    }
    return true;
}

// Stage twiddles W_{Ns R}^{r k} = exp(-2 pi i ((r k) mod L) / L), L = Ns R,
// computed in FP64 from the reduced integer phase, rounded once.
template <typename T>
void build_twiddles(const FftSpec &fs, std::vector<T> &out) {
    int total = 0, Ns = 1;
    for (int s = 0; s < fs.nstages; ++s) {
        total += Ns * (fs.radix[s] - 1);
        Ns *= fs.radix[s];
    }
    out.assign(2 * (size_t)(total > 0 ? total : 1), T(0));
    Ns = 1;
    const double two_pi = 6.283185307179586476925286766559;
    for (int s = 0; s < fs.nstages; ++s) {
        const int R = fs.radix[s];
        const long long L = (long long)Ns * R;
        for (int k = 0; k < Ns; ++k)
            for (int r = 1; r < R; ++r) {
                const long long m = ((long long)r * k) % L;
                const double ang = two_pi * (double)m / (double)L;
                const size_t i = (size_t)fs.twoff[s] + (size_t)k * (R - 1) + (r - 1);
                out[2 * i] = (T)std::cos(ang);
                out[2 * i + 1] = (T)(-std::sin(ang));
            }
        Ns *= R;
    }
}

void block_split(int n, int M, int r, int *start, int *size) {
    const int q = n / M, rem = n % M;
    *size = q + (r < rem ? 1 : 0);
    *start = r * q + (r < rem ? r : rem);
}

// Threads per column (power of two, >= n / kEMax) and columns per tile, while
// the tile fits max_threads threads and the LDS budget.
void choose_tile(int n, int csize, int max_tc, int *tc_log2, int *wpc_log2, int *pitch, size_t *lds,
                 int max_threads = 512) {
    const int emax = csize == 16 ? pf::kEMax / 2 : pf::kEMax;  // elements per thread (F64 halves it)
    int wpc = 1;
    while (wpc * emax < n) wpc <<= 1;
    if (wpc > 1024) wpc = 1024;
    const int p = pf::pidx(n - 1) + 1;
    int tc = 1;
    while (tc * 2 <= max_tc && tc * 2 * wpc <= max_threads && (size_t)(tc * 2) * p * csize <= kLdsBudget) tc <<= 1;
    *tc_log2 = ilog2(tc);
    *wpc_log2 = ilog2(wpc);
    *pitch = p;
    *lds = (size_t)tc * p * csize;
}

int hip_status(hipError_t e) {
    if (e == hipSuccess) return PF_OK;
    if (e == hipErrorOutOfMemory) return PF_ENOMEM;
    return PF_EHIP;
}

int check_impl(int nx, int ny, int nz, const pf_layout *l) {
    if (!l) return PF_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return PF_EINVAL;
    if (!valid_layout_values(l)) return PF_EINVAL;
    const int nxh = nx / 2 + 1;
    // Eq. 2 read as: every rank's block of every pencil is non-empty.
    if (l->m1 > nxh || l->m1 > ny || l->m2 > ny || l->m2 > nz) return PF_EINVAL;
    FftSpec f;
    // under the Chebyshev third transform the z length transformed is 2 (nz - 1), checked below;
    // the empty third transform transforms nothing along z, so nz need not factor
    const bool cheb = l->third == PF_THIRD_CHEB;
    const bool empty = l->third == PF_THIRD_EMPTY;
    if (!factor_length(nx, &f) || !factor_length(ny, &f) || (!cheb && !empty && !factor_length(nz, &f)))
        return PF_EUNSUPPORTED;
    const int maxn = l->precision == PF_F64 ? 4096 : 8192;
    if (nx > maxn || ny > maxn || nz > maxn) return PF_EUNSUPPORTED;
    if (cheb) {  // the DCT runs as a length 2 (nz - 1) transform
        if (nz < 2) return PF_EINVAL;
        if (!factor_length(2 * (nz - 1), &f) || 2 * (nz - 1) > maxn) return PF_EUNSUPPORTED;
    }
    return PF_OK;
}

// Options accepted by pf_check but not built for this grid / combination.
int built_options(int nx, int ny, const pf_layout *l) {
    if (l->math != PF_PLAIN && l->precision != PF_F32) return PF_EUNSUPPORTED;
    if (l->share_only && l->inplace) return PF_EUNSUPPORTED;
    if (l->fused_xy) {
        if (!pf::p2_fused_supported(nx, ny, l->precision) || l->math != PF_PLAIN || l->share_only ||
            l->m1 * l->m2 > 1)
            return PF_EUNSUPPORTED;
    }
    return PF_OK;
}

// The power-of-two kernel serves every side: the padded workspace (whole
// 16-column blocks, 16-byte aligned rows), contiguous lines, and unaligned
// rows (Side::v8).
void set_c2c_common(PassDesc &d, const pf_plan *p, const FftSpec &fs, size_t twoff, int dir, int max_tc,
                    int tuned_tc = 0, bool plain_fft = true, int axis = -1) {
    if (tuned_tc > 0 && tuned_tc < max_tc) max_tc = tuned_tc;
    d.dir = dir;
    d.prec = p->lay.precision;
    PassArgs &a = d.a;
    std::memset(&a, 0, sizeof(a));
    a.fft = fs;
    a.tw = (const char *)p->tw_dev + twoff;
    a.C = p->nxh;
    if (!p->opt.generic_only && pf::p2_supported(fs.n, p->lay.precision) && pf::p2_tc(fs.n) <= max_tc) {
        // compile-time radix plan, persistent blocks (grid set once the tile count is known)
        d.kind = pf::PASS_C2C_P2;
        a.math = pf::p2_has_mfma(fs.n) ? p->lay.math : 0;
        a.tc_log2 = ilog2(pf::p2_tc(fs.n));
        a.wpc_log2 = ilog2(fs.n / 16);
        d.threads = (unsigned)pf::p2_threads(fs.n);
        d.lds = pf::p2_lds_bytes(fs.n, a.math);
        return;
    }
    if (!p->opt.generic_only && p->lay.precision == PF_F64 && plain_fft && pf::p2d_supported(fs.n) &&
        p->B <= max_tc) {
        // FP64 compile-time radix plan: 8 columns (one 128-byte row) per tile, persistent blocks
        d.kind = pf::PASS_C2C_P2;
        a.math = 0;
        a.tc_log2 = ilog2(p->B);
        a.wpc_log2 = ilog2(fs.n / 16);
        d.threads = (unsigned)pf::p2d_threads(fs.n);
        d.lds = pf::p2d_lds_bytes(fs.n);
        return;
    }
    if (axis >= 0 && p->mr[axis] && plain_fft && max_tc >= 16) {
        // compile-time mixed-radix plan: 16 columns per tile, one tile per workgroup
        d.kind = pf::PASS_C2C_MR;
        a.tw = (const char *)p->tw_dev + p->tw_mr[axis];
        a.tc_log2 = 4;
        a.wpc_log2 = 0;
        d.threads = (unsigned)pf::mr_threads_of(fs.n, 0);
        d.lds = pf::mr_lds_bytes(fs.n, 0);
        return;
    }
    d.kind = pf::PASS_C2C;
    choose_tile(fs.n, p->csize, max_tc, &a.tc_log2, &a.wpc_log2, &a.pitch, &d.lds);
    d.threads = 1u << (a.tc_log2 + a.wpc_log2);
}

// Grid of a C2C pass over A * CB tiles: one block per tile, or for the
// persistent power-of-two kernel as many blocks as fit on the device at once.
// Tile traversal order of the power-of-two C2C passes, measured at 1024^3:
// the backward Z pass reads the user's Z-pencil lines (16 lines of a tile are
// ny nz elements apart) and is faster when concurrently resident tiles spread
// over ky (order 1); the forward Z pass, which writes those lines, is faster
// in order 0.
// largest ny for which plans take the transposed backward chain (measured:
// faster up to 512, slower at 1024)
#ifndef PF_BWD_TR_MAX_NY
#define PF_BWD_TR_MAX_NY 512
#endif
// 1: plans that take the transposed backward chain take the forward one too
#ifndef PF_FWD_TR
#define PF_FWD_TR 1
#endif
// 1: Chebyshev plans with the split spectral kernel take the transposed chains
#ifndef PF_CHEB_TR
#define PF_CHEB_TR 1
#endif
#ifndef PF_TILE_ORDER_FZ
#define PF_TILE_ORDER_FZ 0
#endif
#ifndef PF_TILE_ORDER_BZ
#define PF_TILE_ORDER_BZ 1
#endif
#ifndef PF_TILE_ORDER_Y
#define PF_TILE_ORDER_Y 0
#endif
// mixed-radix Z passes: order 1 (ky fastest) measured within 1% of order 0 at
// 480 x 360 x 250, 320^3 and on the 64-transform batch
#ifndef PF_TILE_ORDER_MRZ
#define PF_TILE_ORDER_MRZ 0
#endif
#ifndef PF_XCD_UROWS
#define PF_XCD_UROWS 1
#endif

unsigned c2c_grid(const pf_plan *p, PassDesc &d) {
    const long long tiles = d.a.A * d.a.CB;
    if (d.kind != pf::PASS_C2C_P2) return (unsigned)tiles;
    // side kinds: 1 lines, 0 aligned rows, 2 rows read / written a column at a time
    d.a.inp = (d.a.in_s.sp == 1 && d.a.in_s.sc != 1) ? 1 : d.a.in_s.v8 ? 2 : 0;
    d.a.outp = (d.a.out_s.sp == 1 && d.a.out_s.sc != 1) ? 1 : d.a.out_s.v8 ? 2 : 0;
    // unaligned rows: neighbouring column-block tiles read / write the two
    // halves of shared cache lines; keep them on one XCD (one L2)
    d.a.xcd = d.a.outp == 2 || d.a.inp == 2 ? PF_XCD_UROWS : 0;
    const long long resident = (long long)p->ncu * pf::p2_blocks_per_cu(d);
    return (unsigned)(tiles < resident ? tiles : resident);
}

// Blocked workspace side seen by a C2C pass whose points are sp apart (B for
// Y, zrows B for Z) and whose outer index moves by sa.
Side ws_side(const pf_plan *p, long long sa, long long sp, int tc_log2) {
    Side s;
    s.sa = sa;
    s.sblk = p->kbrows * p->B;
    s.sc = 1;
    s.sp = sp;
    s.cpb = p->B >> tc_log2;
    s.v8 = 0;
    return s;
}

// User Z-pencil side: STRIDE1 [nxh][ny][nz] or [nz][ny][nxh]; outer index y.
Side user_side(const pf_plan *p, long long CB) {
    Side s;
    if (p->lay.stride1) {
        s.sa = p->nz;
        s.sc = (long long)p->ny * p->nz;
        s.sp = 1;
    } else {
        s.sa = p->nxh;
        s.sc = 1;
        s.sp = (long long)p->ny * p->nxh;
    }
    s.sblk = 0;
    s.cpb = CB;
    // [nz][ny][nxh] rows of nxh modes: neither 16-byte aligned nor whole column
    // pairs in general, so the power-of-two kernel reads / writes them one column
    // (8 or 16 bytes) at a time
    s.v8 = p->lay.stride1 || p->csize == 16 ? 0 : 1;
    return s;
}

// m1 x m2 grids: pack the ranks' blocks into the global array before the three
// passes and unpack the result into the ranks' blocks after them (the paper's
// pack / exchange / unpack around each transpose, Sec. 3.3, as on-device
// reorders of whole lines).
void add_remaps(pf_plan *p, int dir) {
    const int rw = p->lay.precision == PF_F64 ? 2 : 1;  // 4-byte words per real
    auto remap = [&](int kind, int gather) {
        PassDesc d;
        std::memset(&d, 0, sizeof(d));
        d.kind = pf::PASS_REMAP;
        d.prec = p->lay.precision;
        pf::RemapArgs &r = d.r;
        r.kind = kind;
        r.gather = gather;
        r.words = kind == pf::REMAP_XPENCIL ? rw : 2 * rw;
        r.nx = p->nx, r.ny = p->ny, r.nz = p->nz, r.nxh = p->nxh, r.m1 = p->lay.m1, r.m2 = p->lay.m2;
        if (kind == pf::REMAP_XPENCIL) r.nlines = (long long)p->ny * p->nz;
        else if (kind == pf::REMAP_ZSTRIDE1) r.nlines = (long long)p->nxh * p->ny;
        else r.nlines = (long long)p->nz * p->ny * p->lay.m1;
        d.blocks = (unsigned)r.nlines;
        d.threads = 256;
        return d;
    };
    const int zkind = p->lay.stride1 ? pf::REMAP_ZSTRIDE1 : pf::REMAP_ZXYZ;
    const double rs = p->lay.precision == PF_F64 ? 8.0 : 4.0;
    const double xb = 2.0 * p->nx * p->ny * p->nz * rs;
    const double zb = 2.0 * 2.0 * p->nxh * p->ny * p->nz * rs;
    for (int i = 3; i >= 1; --i) {
        p->pass[dir][i] = p->pass[dir][i - 1];
        p->pass_names[dir][i] = p->pass_names[dir][i - 1];
        p->pass_bytes[dir][i] = p->pass_bytes[dir][i - 1];
    }
    if (dir == 0) {
        p->pass[0][0] = remap(pf::REMAP_XPENCIL, 1);
        p->pass_names[0][0] = "fwd_pack_x_pencils";
        p->pass_bytes[0][0] = xb;
        p->pass[0][4] = remap(zkind, 0);
        p->pass_names[0][4] = "fwd_unpack_z_pencils";
        p->pass_bytes[0][4] = zb;
    } else {
        p->pass[1][0] = remap(zkind, 1);
        p->pass_names[1][0] = "bwd_pack_z_pencils";
        p->pass_bytes[1][0] = zb;
        p->pass[1][4] = remap(pf::REMAP_XPENCIL, 0);
        p->pass_names[1][4] = "bwd_unpack_x_pencils";
        p->pass_bytes[1][4] = xb;
    }
    p->npass[dir] = 5;
}

// Share-only plan: the local stages of rank (r1, r2) of the m1 x m2 grid at
// their Table 1 shapes (Sec. 2, 3.2), each exchange reduced to the part that
// stays on the rank.  The other ranks' blocks are taken as zero, so the
// forward result is the transform of the input extended by zeros outside the
// rank's X-pencil, restricted to its Z-pencil block, and the backward result
// is the staged C2R of the input extended by zeros outside the rank's
// Z-pencil, restricted to its X-pencil block.  The global-layout workspace W
// and array G hold the blocks at their global positions; zero fills stand in
// for the blocks other ranks would send.
//   forward : fill, X on the rank's lines, Y on its z planes, Z on its ky
//             range, copy of its Z block out of G
//   backward: fill, copy of its Z block into G, Z, Y, zero the modes outside
//             its kx range, X on its lines
void build_share_only(pf_plan *p) {
    const pf_layout &l = p->lay;
    int xs, xl, ys1, yl1, zs2, zl2, ys2, yl2;
    block_split(p->nxh, l.m1, l.r1, &xs, &xl);
    block_split(p->ny, l.m1, l.r1, &ys1, &yl1);
    block_split(p->nz, l.m2, l.r2, &zs2, &zl2);
    block_split(p->ny, l.m2, l.r2, &ys2, &yl2);
    const int B = p->B;
    const int kbA = xs / B, kbB = (xs + xl - 1) / B + 1;  // column blocks [kbA, kbB) hold the rank's modes
    const size_t zplane = (size_t)p->zrows * B, kblock = (size_t)p->kbrows * B;  // complex elements
    const int rw = l.precision == PF_F64 ? 2 : 1;
    const double rs = 4.0 * rw, cs = 2.0 * rs;
    const int ncolsK = std::min(p->nxh, kbB * B) - kbA * B;
    p->so_x = (size_t)zs2 * zplane * p->csize;
    p->so_y = ((size_t)zs2 * zplane + (size_t)kbA * kblock) * p->csize;
    p->so_zw = ((size_t)ys2 * B + (size_t)kbA * kblock) * p->csize;
    p->so_zg = (l.stride1 ? ((size_t)kbA * B * p->ny * p->nz + (size_t)ys2 * p->nz)
                          : ((size_t)kbA * B + (size_t)ys2 * p->nxh)) * p->csize;

    // boxes {z0, z1, kb0, kb1, y0, y1}; bytes: the elements actually zeroed
    auto fill = [&](int nbox, const int (*box)[6], int keep0, int keep1, double *bytes) {
        PassDesc d;
        std::memset(&d, 0, sizeof(d));
        d.kind = pf::PASS_FILL;
        d.prec = l.precision;
        pf::FillArgs &f = d.f;
        f.words = 2 * rw, f.B = B, f.ny = p->ny, f.zrows = p->zrows, f.kbrows = p->kbrows;
        f.keep0 = keep0, f.keep1 = keep1;
        f.nbox = nbox;
        *bytes = 0;
        for (int i = 0; i < nbox; ++i) {
            f.z0[i] = box[i][0], f.z1[i] = box[i][1], f.kb0[i] = box[i][2], f.kb1[i] = box[i][3];
            f.y0[i] = box[i][4], f.y1[i] = box[i][5];
            const double rows = (double)std::max(0, box[i][1] - box[i][0]) * std::max(0, box[i][5] - box[i][4]);
            const int cols = std::max(0, box[i][3] - box[i][2]) * B;
            const int kept = std::max(0, std::min(keep1, box[i][3] * B) - std::max(keep0, box[i][2] * B));
            *bytes += rows * (cols - kept) * cs;
        }
        return d;
    };
    auto box = [&](int to_block) {
        PassDesc d;
        std::memset(&d, 0, sizeof(d));
        d.kind = pf::PASS_BOX;
        d.prec = l.precision;
        pf::BoxArgs &b = d.b;
        b.words = 2 * rw;
        b.to_block = to_block;
        if (l.stride1) {  // G [kx][ky][kz], block [xl][yl2][nz]
            b.st1 = p->nz, b.st2 = (long long)p->ny * p->nz;
            b.o0 = 0, b.o1 = ys2, b.o2 = xs, b.s0 = p->nz, b.s1 = yl2, b.s2 = xl;
        } else {  // G [kz][ky][kx], block [nz][yl2][xl]
            b.st1 = p->nxh, b.st2 = (long long)p->ny * p->nxh;
            b.o0 = xs, b.o1 = ys2, b.o2 = 0, b.s0 = xl, b.s1 = yl2, b.s2 = p->nz;
        }
        return d;
    };
    for (int dir = 0; dir < 2; ++dir) {
        PassDesc x = p->pass[dir][dir == 0 ? 0 : 2];
        PassDesc y = p->pass[dir][1];
        PassDesc z = p->pass[dir][dir == 0 ? 2 : 0];
        // X on the rank's lines: y_local < yl1 in each of its zl2 planes
        x.a.lines = (long long)yl1 * zl2;
        x.a.ny = yl1;
        x.a.y0 = ys1;
        if (x.kind == pf::PASS_R2C_P2 || x.kind == pf::PASS_C2R_P2) {
            const long long tl = pf::p2x_tile_lines(x.prec, 0);
            const long long tiles = (x.a.lines + tl - 1) / tl;
            const long long resident = (long long)p->ncu * pf::p2_blocks_per_cu(x);
            x.blocks = (unsigned)std::min(tiles, resident);
        } else {
            const long long pairs = (x.a.lines + 1) / 2, tcx = 1LL << x.a.tc_log2;
            x.blocks = (unsigned)((pairs + tcx - 1) / tcx);
        }
        // Y on the rank's z planes and the column blocks of its modes
        y.a.A = zl2;
        y.a.CB = (long long)(kbB - kbA) * (B >> y.a.tc_log2);
        y.a.C = p->nxh - kbA * B;
        y.blocks = c2c_grid(p, y);
        // Z on the rank's ky range and the same column blocks
        z.a.A = yl2;
        z.a.CB = y.a.CB;
        z.a.C = y.a.C;
        z.blocks = c2c_grid(p, z);
        const double xbytes = (double)x.a.lines * (p->nx * rs + p->nxh * cs);
        const double ybytes = 2.0 * zl2 * p->ny * ncolsK * cs;
        const double zbytes = 2.0 * yl2 * p->nz * ncolsK * cs;
        const double bbytes = 2.0 * xl * yl2 * p->nz * cs;
        if (dir == 0) {
            const int fb[4][6] = {{zs2, zs2 + zl2, kbA, kbB, 0, ys1},
                                  {zs2, zs2 + zl2, kbA, kbB, ys1 + yl1, p->ny},
                                  {0, zs2, kbA, kbB, ys2, ys2 + yl2},
                                  {zs2 + zl2, p->nz, kbA, kbB, ys2, ys2 + yl2}};
            double fbytes;
            p->pass[0][0] = fill(4, fb, 0, 0, &fbytes);
            p->pass[0][1] = x;
            p->pass[0][2] = y;
            p->pass[0][3] = z;
            p->pass[0][4] = box(1);
            const char *names[] = {"share_fill", "share_x_r2c", "share_y_c2c", "share_z_c2c", "share_extract_z"};
            const double bytes[] = {fbytes, xbytes, ybytes, zbytes, bbytes};
            for (int i = 0; i < 5; ++i) p->pass_names[0][i] = names[i], p->pass_bytes[0][i] = bytes[i];
            p->npass[0] = 5;
        } else {
            const int fb[2][6] = {{zs2, zs2 + zl2, kbA, kbB, 0, ys2}, {zs2, zs2 + zl2, kbA, kbB, ys2 + yl2, p->ny}};
            // modes outside [xs, xs + xl) of the rank's X-pencil rows: whole column
            // blocks below kbA and from kbB on, and the two partial blocks at the ends
            const int lastA = kbB - 1;
            const int mb[4][6] = {{zs2, zs2 + zl2, 0, kbA, ys1, ys1 + yl1},
                                  {zs2, zs2 + zl2, kbA, kbA + 1, ys1, ys1 + yl1},
                                  {zs2, zs2 + zl2, lastA > kbA ? lastA : kbA, lastA > kbA ? kbB : kbA, ys1, ys1 + yl1},
                                  {zs2, zs2 + zl2, kbB, p->nkb, ys1, ys1 + yl1}};
            double fbytes, mbytes;
            p->pass[1][0] = fill(2, fb, 0, 0, &fbytes);
            p->pass[1][1] = box(0);
            p->pass[1][2] = z;
            p->pass[1][3] = y;
            p->pass[1][4] = fill(4, mb, xs, xs + xl, &mbytes);
            p->pass[1][5] = x;
            const char *names[] = {"share_fill", "share_insert_z", "share_z_c2c", "share_y_c2c", "share_mask_kx",
                                   "share_x_c2r"};
            const double bytes[] = {fbytes, bbytes, zbytes, ybytes, mbytes, xbytes};
            for (int i = 0; i < 6; ++i) p->pass_names[1][i] = names[i], p->pass_bytes[1][i] = bytes[i];
            p->npass[1] = 6;
        }
    }
}

// Fused plans: the X and Y passes of each direction become one pass (the
// first forward, the last backward); the Z passes stay.  Items: 512 threads'
// worth of 16-line X tiles or Y tiles (z, column block) of one plane.
constexpr int kFusedLag = 2;         // planes of producer work a queue runs ahead of its consumer work
constexpr long long kFusedSpin = 1LL << 22;  // polls before a wait gives up (a few seconds)

void build_fused(pf_plan *p) {
    for (int dir = 0; dir < 2; ++dir) {
        const PassDesc &x = p->pass[dir][dir == 0 ? 0 : 2];
        const PassDesc &y = p->pass[dir][1];
        const PassDesc z = p->pass[dir][dir == 0 ? 2 : 0];
        pf::FusedArgs &f = p->fxy[dir];
        std::memset(&f, 0, sizeof(f));
        f.x = x.a;
        f.y = y.a;
        f.ctl = p->ctl;
        f.nq = p->fused_nq;
        f.lag = kFusedLag;
        f.nz = p->nz;
        f.xtiles = p->ny / 16;
        f.ytiles = (int)y.a.CB;
        const int xt = pf::p2_fused_tiles_per_item(p->nx, 1), yt = pf::p2_fused_tiles_per_item(p->ny, 0);
        f.xitems = (f.xtiles + xt - 1) / xt;
        f.yitems = (f.ytiles + yt - 1) / yt;
        f.spin_limit = kFusedSpin;
        PassDesc d;
        std::memset(&d, 0, sizeof(d));
        d.kind = pf::PASS_FUSED_XY;
        d.dir = dir == 0 ? -1 : 1;
        d.prec = p->lay.precision;
        d.blocks = p->fused_blocks;
        d.threads = 512;
        d.lds = pf::p2_fused_lds_bytes(p->nx, p->ny);
        const double xb = p->pass_bytes[dir][dir == 0 ? 0 : 2];  // N s + M 2s
        if (dir == 0) {
            p->pass[0][0] = d;
            p->pass[0][1] = z;
            p->pass_names[0][0] = "fwd_xy_fused";
            p->pass_names[0][1] = "fwd_z_c2c";
            p->pass_bytes[0][1] = p->pass_bytes[0][2];
            p->pass_bytes[0][0] = xb;
        } else {
            p->pass[1][1] = d;
            p->pass_names[1][1] = "bwd_yx_fused";
            p->pass_bytes[1][1] = xb;
        }
        p->npass[dir] = 2;
    }
}

void build_passes(pf_plan *p) {
    const long long zstride = p->zrows * p->B;  // complex elements between z planes of W
    const double rs = p->lay.precision == PF_F64 ? 8.0 : 4.0;
    const double N = (double)p->nx * p->ny * p->nz;
    const double M = (double)p->nxh * p->ny * p->nz;
    for (int dir = 0; dir < 2; ++dir) {
        const int sgn = dir == 0 ? -1 : 1;
        // X stage
        PassDesc x;
        std::memset(&x, 0, sizeof(x));
        x.kind = dir == 0 ? pf::PASS_R2C_X : pf::PASS_C2R_X;
        x.dir = sgn;
        x.prec = p->lay.precision;
        x.a.fft = p->fx;
        x.a.tw = (const char *)p->tw_dev + p->tw_off[0];
        const int xmax = p->opt.tile[0] > 0 && p->opt.tile[0] < 64 ? p->opt.tile[0] : 64;
        // X tiles of at most 256 threads: more, smaller blocks per CU measured
        // 3-9% faster on the generic X passes (the Y / Z passes keep 512)
        choose_tile(p->nx, p->csize, xmax, &x.a.tc_log2, &x.a.wpc_log2, &x.a.pitch, &x.lds, 256);
        x.threads = 1u << (x.a.tc_log2 + x.a.wpc_log2);
        x.a.lines = (long long)p->ny * p->nz;
        x.a.ld_real = p->nx;
        x.a.ny = p->ny;
        x.a.nkb = p->nkb;
        x.a.b_log2 = p->b_log2;
        x.a.nxh = p->nxh;
        x.a.zrows = p->zrows;
        x.a.kbrows = p->kbrows;
        x.a.y0 = 0;
        const long long pairs = (x.a.lines + 1) / 2;
        const long long tcx = 1LL << x.a.tc_log2;
        x.blocks = (unsigned)((pairs + tcx - 1) / tcx);
        if (p->mr[0] && xmax >= 16) {  // compile-time mixed-radix plan, mr_x_pairs() line pairs per tile
            const int xp = pf::mr_x_pairs();
            x.kind = dir == 0 ? pf::PASS_R2C_MR : pf::PASS_C2R_MR;
            x.a.tw = (const char *)p->tw_dev + p->tw_mr[0];
            x.a.tc_log2 = ilog2(xp);
            x.a.wpc_log2 = 0;
            x.threads = (unsigned)pf::mr_threads_of(p->nx, 1);
            x.lds = pf::mr_lds_bytes(p->nx, 1);
            x.blocks = (unsigned)((pairs + xp - 1) / xp);
        }
        if (p->fast_x) {  // half-length complex transform, 16 (FP64: 8) lines per tile, persistent blocks
            x.kind = dir == 0 ? pf::PASS_R2C_P2 : pf::PASS_C2R_P2;
            x.a.fft = p->fxh;
            x.a.math = pf::p2_has_mfma(p->nx / 2) && p->lay.precision == PF_F32 ? p->lay.math : 0;
            x.a.tw = (const char *)p->tw_dev + p->tw_off[3];
            x.threads = (unsigned)pf::p2x_threads(p->nx, x.prec, 0);
            x.lds = pf::p2x_lds_bytes(p->nx, x.a.math, x.prec, 0);
            const long long tl = pf::p2x_tile_lines(x.prec, 0);
            const long long tiles = (x.a.lines + tl - 1) / tl;
            const long long resident = (long long)p->ncu * pf::p2_blocks_per_cu(x);
            x.blocks = (unsigned)(tiles < resident ? tiles : resident);
        }
        // Y stage: in place on the workspace, tile (z, column block)
        PassDesc y;
        set_c2c_common(y, p, p->fy, p->tw_off[1], sgn, p->B, p->opt.tile[1], true, 1);
        y.a.in_s = ws_side(p, zstride, p->B, y.a.tc_log2);
        y.a.out_s = y.a.in_s;
        y.a.A = p->nz;
        y.a.CB = (long long)p->nkb * (p->B >> y.a.tc_log2);
        y.a.tile_order = PF_TILE_ORDER_Y;
        y.blocks = c2c_grid(p, y);
        // Z stage: tile (y, column block); with the empty third transform
        // (Sec. 3.1) a zero-stage plan, so the pass is the reorder alone
        PassDesc z;
        const bool empty = p->lay.third == PF_THIRD_EMPTY;
        FftSpec fz = p->fz;
        if (empty) fz.nstages = 0;
        const bool cheb = p->lay.third == PF_THIRD_CHEB;  // type-I DCT by the even extension
        set_c2c_common(z, p, fz, p->tw_off[2], sgn, p->B, p->opt.tile[2], !empty && !cheb, 2);
        if (cheb) z.a.cheb = p->nz;
        if (cheb && z.kind == pf::PASS_C2C_P2) z.a.math = 4;  // mirrored loads, the first nz points stored
        if (empty && z.kind == pf::PASS_C2C_P2) z.a.math = 3;  // the power-of-two kernel's reorder-only form
        z.a.A = p->ny;
        z.a.CB = (long long)p->nkb * (p->B >> z.a.tc_log2);
        const Side wsz = ws_side(p, p->B, zstride, z.a.tc_log2);
        const Side usr = user_side(p, z.a.CB);
        z.a.in_s = dir == 0 ? wsz : usr;
        z.a.out_s = dir == 0 ? usr : wsz;
        // a backward Z pass reading the unaligned [nz][ny][nxh] rows does best
        // walking column blocks first, so that neighbouring tiles (on one XCD)
        // share the cache lines the rows straddle
        z.a.tile_order = dir == 0 ? PF_TILE_ORDER_FZ : (p->lay.stride1 ? PF_TILE_ORDER_BZ : 0);
        if (z.kind == pf::PASS_C2C_MR) z.a.tile_order = PF_TILE_ORDER_MRZ;
        z.blocks = c2c_grid(p, z);

        if ((dir == 1 && p->bwd_tr) || (dir == 0 && p->fwd_tr)) {
            // Z: 16 adjacent ky lines of one kx of the Z-pencil per tile (one
            // contiguous run) <-> rows (z, kx, ky block) of W' (backward: lines in,
            // rows out; forward: rows in, lines out)
            PassDesc z2;
            set_c2c_common(z2, p, fz, p->tw_off[2], sgn, p->B, p->opt.tile[2], !cheb, 2);
            if (cheb) z2.a.cheb = p->nz;
            if (cheb && z2.kind == pf::PASS_C2C_P2) z2.a.math = 4;  // the even extension, as above
            const long long tcz = 1LL << z2.a.tc_log2;
            z2.a.A = p->nxh;
            z2.a.CB = (p->ny + tcz - 1) / tcz;
            z2.a.C = p->ny;
            Side zi, zo;
            zi.sa = (long long)p->ny * p->nz, zi.sblk = 0, zi.sc = p->nz, zi.sp = 1, zi.cpb = z2.a.CB, zi.v8 = 0;
            zo.sa = p->ny, zo.sblk = 0, zo.sc = 1, zo.sp = (long long)p->nxh * p->ny, zo.cpb = z2.a.CB, zo.v8 = 0;
            z2.a.in_s = dir == 1 ? zi : zo;
            z2.a.out_s = dir == 1 ? zo : zi;
            z2.a.tile_order = 0;
            z2.blocks = c2c_grid(p, z2);
            // Y: in place along the contiguous ky lines of W', 16 adjacent kx per tile
            PassDesc y2;
            set_c2c_common(y2, p, p->fy, p->tw_off[1], sgn, p->B, p->opt.tile[1], true, 1);
            const long long tcy = 1LL << y2.a.tc_log2;
            y2.a.A = p->nz;
            y2.a.CB = (p->nxh + tcy - 1) / tcy;
            y2.a.C = p->nxh;
            Side yl;
            yl.sa = (long long)p->nxh * p->ny, yl.sblk = 0, yl.sc = p->ny, yl.sp = 1, yl.cpb = y2.a.CB, yl.v8 = 0;
            y2.a.in_s = yl;
            y2.a.out_s = yl;
            y2.a.tile_order = 0;
            y2.blocks = c2c_grid(p, y2);
            // X: rows of W' hold a tile's 16 lines at one mode (its own kernel, for FP64
            // with 16-line tiles: the grid again)
            x.a.xtr = 1;
            x.a.zrows = (long long)p->nxh * p->ny;
            x.a.kbrows = p->ny;
            x.threads = (unsigned)pf::p2x_threads(p->nx, x.prec, 1);
            x.lds = pf::p2x_lds_bytes(p->nx, x.a.math, x.prec, 1);
            const long long xtl = pf::p2x_tile_lines(x.prec, 1);
            const long long xtiles = (x.a.lines + xtl - 1) / xtl;
            const long long xres = (long long)p->ncu * pf::p2_blocks_per_cu(x);
            x.blocks = (unsigned)(xtiles < xres ? xtiles : xres);
            z = z2;
            y = y2;
        }
        const double cbytes = M * 2 * rs;
        if (dir == 0) {
            p->pass[0][0] = x;
            p->pass[0][1] = y;
            p->pass[0][2] = z;
            p->pass_names[0][0] = "fwd_x_r2c";
            p->pass_names[0][1] = "fwd_y_c2c";
            p->pass_names[0][2] = "fwd_z_c2c";
            p->pass_bytes[0][0] = N * rs + cbytes;
            p->pass_bytes[0][1] = 2 * cbytes;
            p->pass_bytes[0][2] = 2 * cbytes;
        } else {
            p->pass[1][0] = z;
            p->pass[1][1] = y;
            p->pass[1][2] = x;
            p->pass_names[1][0] = "bwd_z_c2c";
            p->pass_names[1][1] = "bwd_y_c2c";
            p->pass_names[1][2] = "bwd_x_c2r";
            p->pass_bytes[1][0] = 2 * cbytes;
            p->pass_bytes[1][1] = 2 * cbytes;
            p->pass_bytes[1][2] = N * rs + cbytes;
        }
        p->npass[dir] = 3;
        if (p->blocked) add_remaps(p, dir);
        if (dir == 0 && cheb && z.kind == pf::PASS_C2C_P2 && p->lay.precision == PF_F32 && !p->blocked && !p->share) {
            // fused spectral step: the forward Z pass's tiles, W on both sides (on the
            // transposed workspace: its rows of 16 ky at one kx, and a.xtr = 1)
            PassDesc f = z;
            f.a.in_s = f.a.out_s = p->fwd_tr ? z.a.in_s : wsz;
            f.a.xtr = p->fwd_tr ? 1 : 0;
            f.a.inp = f.a.outp = 0;
            f.a.tile_order = 0;
            f.a.xcd = 0;
            f.lds = pf::p2_lds_bytes(fz.n, 0);
            const long long tiles = f.a.A * f.a.CB;
            const long long resident = (long long)p->ncu * pf::p2_spec_blocks_per_cu(fz.n, f.threads, f.lds);
            f.blocks = (unsigned)(tiles < resident ? tiles : resident);
            if (p->spec_sr) {  // the split type-I DCT: one tile per workgroup
                f.a.math = 5;
                f.a.tw = (const char *)p->tw_dev + p->tw_dct;
                f.threads = pf::p2_spec_sr_threads(p->nz);
                f.lds = pf::p2_spec_sr_lds_bytes(p->nz);
                f.blocks = (unsigned)tiles;
            }
            p->spec = f;
            p->spec_fused = true;
        }
    }
    if (p->share) build_share_only(p);
    if (p->fused) build_fused(p);
}

EventPair take_events(pf_plan *p) {
    if (!p->pool.empty()) {
        EventPair e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    EventPair e{nullptr, nullptr};
    if (hipEventCreate(&e.start) != hipSuccess) e.start = nullptr;
    if (hipEventCreate(&e.stop) != hipSuccess) e.stop = nullptr;
    return e;
}

void release_timing(pf_plan *p) {
    for (int d = 0; d < 2; ++d)
        for (int i = 0; i < kPasses; ++i) {
            for (auto &e : p->tim[d][i].used) p->pool.push_back(e);
            p->tim[d][i].used.clear();
        }
}

// Set the buffers of pass i of direction dir and enqueue it.  untimed: record
// no events even with timing on (the no-allocation entry point creates none).
int run_one(pf_plan *p, int dir, int i, const void *in, void *out, hipStream_t s, bool untimed = false) {
    PassDesc d = p->pass[dir][i];
    d.a.in = in;
    d.a.out = out;
    d.r.src = in;
    d.r.dst = out;
    d.f.w = out;
    d.b.src = in;
    d.b.dst = out;
    EventPair ev{nullptr, nullptr};
    bool timed = false;
    if (p->timing && !untimed) {
        ev = take_events(p);
        timed = ev.start && ev.stop && hipEventRecord(ev.start, s) == hipSuccess;
    }
    hipError_t e;
    if (d.kind == pf::PASS_FUSED_XY) {  // X reads / writes the user side, Y runs in place on the workspace
        pf::FusedArgs f = p->fxy[dir];
        if (dir == 0) {
            f.x.in = in, f.x.out = out;
            f.y.in = out, f.y.out = out;
        } else {  // in is the workspace, transformed in place along y first
            f.y.in = in, f.y.out = const_cast<void *>(in);
            f.x.in = in, f.x.out = out;
        }
        e = pf::p2_fused_launch(f, dir == 0, p->nx, p->ny, d.blocks, s);
    } else {
        e = pf::launch_pass(d, s);
    }
    // a pass whose events could not be recorded is left out of the timing
    if (timed && hipEventRecord(ev.stop, s) == hipSuccess)
        p->tim[dir][i].used.push_back(ev);
    else if (p->timing && !untimed)
        p->pool.push_back(ev);
    return hip_status(e);
}

bool aligned16(const void *ptr) { return ((uintptr_t)ptr & 15u) == 0; }

int check_args(const pf_plan *p, const void *in, const void *out) {
    if (!p || !in || !out) return PF_EINVAL;
    if (!aligned16(in) || !aligned16(out)) return PF_EALIGN;
    if (p->lay.inplace && in != out) return PF_EALIAS;
    if (!p->lay.inplace && in == out) return PF_EALIAS;
    return PF_OK;
}

int check_call(const pf_plan *p, const void *in, const void *out) {
    const int rc = check_args(p, in, out);
    if (rc) return rc;
    if (!p->ws) return PF_EWORKSPACE;
    return PF_OK;
}

// The pass chain of one direction with workspace ws (the plan's, or the
// no-allocation entry point's static scratch; untimed for the latter).
int run_chain_ws(pf_plan *p, int dir, const void *in, void *out, void *ws, hipStream_t s, bool untimed) {
    if (p->share) {
        char *w = (char *)ws, *g = (char *)ws + p->w_bytes;
        int r;
        if (dir == 0) {
            r = run_one(p, 0, 0, nullptr, w, s, untimed);
            if (!r) r = run_one(p, 0, 1, in, w + p->so_x, s, untimed);
            if (!r) r = run_one(p, 0, 2, w + p->so_y, w + p->so_y, s, untimed);
            if (!r) r = run_one(p, 0, 3, w + p->so_zw, g + p->so_zg, s, untimed);
            if (!r) r = run_one(p, 0, 4, g, out, s, untimed);
        } else {
            r = run_one(p, 1, 0, nullptr, w, s, untimed);
            if (!r) r = run_one(p, 1, 1, in, g, s, untimed);
            if (!r) r = run_one(p, 1, 2, g + p->so_zg, w + p->so_zw, s, untimed);
            if (!r) r = run_one(p, 1, 3, w + p->so_y, w + p->so_y, s, untimed);
            if (!r) r = run_one(p, 1, 4, nullptr, w, s, untimed);
            if (!r) r = run_one(p, 1, 5, w + p->so_x, out, s, untimed);
        }
        return r;
    }
    if (p->fused) {  // pass 0: user -> workspace; pass 1: workspace -> user
        int r = run_one(p, dir, 0, in, ws, s, untimed);
        if (!r) r = run_one(p, dir, 1, ws, out, s, untimed);
        return r;
    }
    if (!p->blocked) {
        // pass 0: user -> workspace; pass 1: workspace in place; pass 2: workspace -> user
        int r = run_one(p, dir, 0, in, ws, s, untimed);
        if (!r) r = run_one(p, dir, 1, ws, ws, s, untimed);
        if (!r) r = run_one(p, dir, 2, ws, out, s, untimed);
        return r;
    }
    // pack: user blocks -> global array G; then G -> W, W in place, W -> G; unpack: G -> user blocks
    void *g = (char *)ws + p->w_bytes;
    int r = run_one(p, dir, 0, in, g, s, untimed);
    if (!r) r = run_one(p, dir, 1, g, ws, s, untimed);
    if (!r) r = run_one(p, dir, 2, ws, ws, s, untimed);
    if (!r) r = run_one(p, dir, 3, ws, g, s, untimed);
    if (!r) r = run_one(p, dir, 4, g, out, s, untimed);
    return r;
}

int run_chain(pf_plan *p, int dir, const void *in, void *out, void *stream) {
    const int rc = check_call(p, in, out);
    if (rc) return rc;
    return run_chain_ws(p, dir, in, out, p->ws, (hipStream_t)stream, false);
}

// ---- static scratch for the no-allocation entry point ----------------------
// One array per device, allocated with the library's code object and held
// until the process ends.  Host code never uses its name as an address: the
// device address comes from hipGetSymbolAddress, once per device (at plan
// creation, or at the entry point's first call on a device).
constexpr size_t kScratchBytes = PF_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices];  // device address of `scratch` per device, nullptr until looked up

// Device address of the current device's scratch array (nullptr on failure).
void *scratch_address() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        scratch_ptr[dev] = ptr;
    }
    return scratch_ptr[dev];
}

}  // namespace

extern "C" {

void pf_layout_init(pf_layout *l) {
    if (!l) return;
    std::memset(l, 0, sizeof(*l));
    l->m1 = 1;
    l->m2 = 1;
    l->stride1 = 1;
    l->precision = PF_F32;
    l->math = PF_PLAIN;
    l->third = PF_THIRD_FFT;
}

int pf_check(int nx, int ny, int nz, const pf_layout *l) { return check_impl(nx, ny, nz, l); }

int pf_query_dims(int nx, int ny, int nz, const pf_layout *l, int pencil, int r1, int r2, int start[3],
                  int size[3], int order[3]) {
    const int rc = check_impl(nx, ny, nz, l);
    if (rc) return rc;
    if (!start || !size || !order) return PF_EINVAL;
    if (r1 < 0 || r1 >= l->m1 || r2 < 0 || r2 >= l->m2) return PF_EINVAL;
    const int nxh = nx / 2 + 1;
    int s0, n0, s1, n1, s2, n2;
    switch (pencil) {
        case PF_PENCIL_X:  // X whole, Y over M1, Z over M2; order XYZ
            s0 = 0, n0 = nx;
            block_split(ny, l->m1, r1, &s1, &n1);
            block_split(nz, l->m2, r2, &s2, &n2);
            order[0] = 0, order[1] = 1, order[2] = 2;
            break;
        case PF_PENCIL_Y:  // X modes over M1, Y whole, Z over M2; YXZ or XYZ
            block_split(nxh, l->m1, r1, &s0, &n0);
            s1 = 0, n1 = ny;
            block_split(nz, l->m2, r2, &s2, &n2);
            if (l->stride1)
                order[0] = 1, order[1] = 0, order[2] = 2;
            else
                order[0] = 0, order[1] = 1, order[2] = 2;
            break;
        case PF_PENCIL_Z:  // X modes over M1, Y over M2, Z whole; ZYX or XYZ
            block_split(nxh, l->m1, r1, &s0, &n0);
            block_split(ny, l->m2, r2, &s1, &n1);
            s2 = 0, n2 = nz;
            if (l->stride1)
                order[0] = 2, order[1] = 1, order[2] = 0;
            else
                order[0] = 0, order[1] = 1, order[2] = 2;
            break;
        default:
            return PF_EINVAL;
    }
    start[0] = s0, start[1] = s1, start[2] = s2;
    size[0] = n0, size[1] = n1, size[2] = n2;
    return PF_OK;
}

static int plan_create(int nx, int ny, int nz, const pf_layout *l, const PlanOpts &o, pf_plan **out) {
    if (!out) return PF_EINVAL;
    *out = nullptr;
    int rc = check_impl(nx, ny, nz, l);
    if (rc) return rc;
    rc = built_options(nx, ny, l);
    if (rc) return rc;
    pf_plan *p = new (std::nothrow) pf_plan();
    if (!p) return PF_ENOMEM;
    p->nx = nx, p->ny = ny, p->nz = nz, p->nxh = nx / 2 + 1;
    p->lay = *l;
    p->opt = o;
    p->csize = l->precision == PF_F64 ? 16 : 8;
    p->B = 128 / p->csize;
    p->b_log2 = ilog2(p->B);
    p->nkb = (p->nxh + p->B - 1) / p->B;
    // W is [z][kb][y][B]: the rows of one (z, kb) are contiguous in y.  (The
    // [kb][z][y][B] order, which brings a Z tile's rows 16 times closer
    // together, measured slower on both Z passes at 1024^3.)
    p->zrows = (long long)p->nkb * ny;
    p->kbrows = (long long)ny;
    factor_length(nx, &p->fx, o.radix_order[0]);
    factor_length(ny, &p->fy, o.radix_order[1]);
    if (!factor_length(l->third == PF_THIRD_CHEB ? 2 * (nz - 1) : nz, &p->fz, o.radix_order[2])) {
        // only the empty third transform gets here (check_impl): an nz that does not
        // factor needs no z plan -- zero stages, no twiddles.  Such lengths are never
        // powers of two, so the pass is the generic kernel, which reads no twiddles
        // at zero stages (the power-of-two reorder form copies a full table).
        std::memset(&p->fz, 0, sizeof(p->fz));
        p->fz.n = nz;
    }

    // twiddle tables, one allocation, each table 256-byte aligned
    std::vector<unsigned char> host;
    const FftSpec *specs[3] = {&p->fx, &p->fy, &p->fz};
    for (int i = 0; i < 3; ++i) {
        p->tw_off[i] = host.size();
        if (l->precision == PF_F64) {
            std::vector<double> t;
            build_twiddles<double>(*specs[i], t);
            const unsigned char *b = reinterpret_cast<const unsigned char *>(t.data());
            host.insert(host.end(), b, b + t.size() * sizeof(double));
        } else {
            std::vector<float> t;
            build_twiddles<float>(*specs[i], t);
            const unsigned char *b = reinterpret_cast<const unsigned char *>(t.data());
            host.insert(host.end(), b, b + t.size() * sizeof(float));
        }
        host.resize((host.size() + 255) & ~(size_t)255, 0);
    }
    p->fast_x = !o.generic_only && pf::p2x_supported(nx, l->precision);
    p->tw_off[3] = host.size();
    if (p->fast_x) {
        // [M-point stage table (M - 1)][pad][W_nx^k, k = 0 .. M], M = nx / 2
        const int M = nx / 2;
        factor_length(M, &p->fxh);
        auto split_table = [&](auto zero) {
            typedef decltype(zero) R;
            std::vector<R> t;
            build_twiddles<R>(p->fxh, t);
            t.resize(2 * (size_t)(2 * M + 1), zero);
            const double two_pi = 6.283185307179586476925286766559;
            for (int k = 0; k <= M; ++k) {
                const double ang = two_pi * (double)k / (double)nx;
                t[2 * (size_t)(M + k)] = (R)std::cos(ang);
                t[2 * (size_t)(M + k) + 1] = (R)(-std::sin(ang));
            }
            const unsigned char *b = reinterpret_cast<const unsigned char *>(t.data());
            host.insert(host.end(), b, b + t.size() * sizeof(R));
        };
        if (l->precision == PF_F64) split_table(0.0);
        else split_table(0.f);
        host.resize((host.size() + 255) & ~(size_t)255, 0);
    }
    // mixed-radix tables W_n^m, m < n (FP32 plain transforms; the Chebyshev and
    // empty third transforms keep the runtime-radix kernel)
    const int axis_n[3] = {nx, ny, nz};
    for (int i = 0; i < 3; ++i) {
        p->mr[i] = !o.no_mr && pf::mr_supported(axis_n[i], l->precision) && !(i == 0 && p->fast_x) &&
                   !(i == 2 && l->third != PF_THIRD_FFT);
        p->tw_mr[i] = 0;
        if (!p->mr[i]) continue;
        p->tw_mr[i] = host.size();
        std::vector<float> t(2 * (size_t)axis_n[i]);
        const double two_pi = 6.283185307179586476925286766559;
        for (int m = 0; m < axis_n[i]; ++m) {
            const double ang = two_pi * (double)m / (double)axis_n[i];
            t[2 * (size_t)m] = (float)std::cos(ang);
            t[2 * (size_t)m + 1] = (float)(-std::sin(ang));
        }
        const unsigned char *b = reinterpret_cast<const unsigned char *>(t.data());
        host.insert(host.end(), b, b + t.size() * sizeof(float));
        host.resize((host.size() + 255) & ~(size_t)255, 0);
    }
    // the split type-I DCT of the fused spectral step (FP32, nz = L + 1 = 257)
    p->spec_sr = !o.no_spec_sr && !o.generic_only && l->third == PF_THIRD_CHEB && l->precision == PF_F32 &&
                 pf::p2_spec_sr_supported(nz);
    p->tw_dct = 0;
    if (p->spec_sr) {
        const int L = nz - 1, M = L / 2;
        FftSpec fl, fm;
        factor_length(L, &fl);
        factor_length(M, &fm);
        std::vector<float> tl, tm;
        build_twiddles<float>(fl, tl);
        build_twiddles<float>(fm, tm);
        std::vector<float> t(2 * (size_t)(L + 2 * M), 0.f);
        std::copy(tl.begin(), tl.begin() + 2 * (L - 1), t.begin());
        std::copy(tm.begin(), tm.begin() + 2 * (M - 1), t.begin() + 2 * L);
        const double two_pi = 6.283185307179586476925286766559;
        for (int k = 0; k < M; ++k) {  // W_{4M}^k
            const double ang = two_pi * (double)k / (double)(4 * M);
            t[2 * (size_t)(L + M + k)] = (float)std::cos(ang);
            t[2 * (size_t)(L + M + k) + 1] = (float)(-std::sin(ang));
        }
        p->tw_dct = host.size();
        const unsigned char *b = reinterpret_cast<const unsigned char *>(t.data());
        host.insert(host.end(), b, b + t.size() * sizeof(float));
        host.resize((host.size() + 255) & ~(size_t)255, 0);
    }
    hipError_t e = hipMalloc(&p->tw_dev, host.size());
    if (e != hipSuccess) {
        delete p;
        return hip_status(e);
    }
    e = hipMemcpy(p->tw_dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = pf::prepare_kernels(pf::kMaxLds);
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, dev);
    for (int n : {ny, p->fz.n}) {
        if (e == hipSuccess && pf::p2_supported(n, l->precision)) e = pf::p2_prepare(n);
        if (e == hipSuccess && l->precision == PF_F64 && !o.generic_only && pf::p2d_supported(n)) e = pf::p2d_prepare(n);
    }
    const bool cheb_p2 = l->third == PF_THIRD_CHEB && !o.generic_only && pf::p2_supported(p->fz.n, l->precision);
    if (e == hipSuccess && cheb_p2) e = pf::p2_spec_prepare(p->fz.n);
    if (e == hipSuccess && p->fast_x) e = pf::p2x_prepare(nx, l->precision);
    if (e != hipSuccess) {
        (void)hipFree(p->tw_dev);
        delete p;
        return hip_status(e);
    }
    // the no-allocation entry point's scratch on this device: looked up here so
    // that its first call does not have to
    if (e == hipSuccess && !scratch_address()) e = hipErrorInvalidSymbol;
    if (e != hipSuccess) {
        (void)hipFree(p->tw_dev);
        delete p;
        return hip_status(e);
    }
    p->fused = l->fused_xy != 0;
    if (e == hipSuccess && p->fused) {
        e = pf::p2_fused_prepare(nx, ny);
        int nb = 0;
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pf::p2_fused_symbol(nx, ny, 1), 512,
                                                             pf::p2_fused_lds_bytes(nx, ny));
        p->fused_blocks = (unsigned)(p->ncu * (nb > 0 ? nb : 1));
        // one queue per XCD; the launch's workgroups must cover XCDs 0 .. nq-1
        if (e == hipSuccess) e = pf::p2_xcd_queues(p->fused_blocks, &p->fused_nq);
        if (e == hipSuccess && p->fused_nq == 0) {
            (void)hipFree(p->tw_dev);
            delete p;
            return PF_EUNSUPPORTED;
        }
        const size_t n = (size_t)p->fused_nq + nz + 1;
        if (e == hipSuccess) e = hipMalloc(&p->ctl, n * sizeof(unsigned));
        if (e == hipSuccess) e = hipMemset(p->ctl, 0, n * sizeof(unsigned));
        if (e != hipSuccess) {
            if (p->ctl) (void)hipFree(p->ctl);
            (void)hipFree(p->tw_dev);
            delete p;
            return hip_status(e);
        }
    }
    p->share = l->share_only != 0;
    p->blocked = !p->share && l->m1 * l->m2 > 1;
    p->w_bytes = ((size_t)p->nz * p->nkb * p->ny * p->B * p->csize + 255) & ~(size_t)255;
    p->ws_bytes = p->w_bytes;
    // (ny a multiple of the X tile's 16 lines, so that a row of the transposed
    // workspace holds one tile's lines at one mode)
    // (Chebyshev plans where the fused spectral step has the split DCT, whose
    // kernel also runs on the transposed rows)
    p->bwd_tr = !o.no_bwd_tr && p->fast_x && l->stride1 && !p->share && !p->blocked && !p->fused &&
                (l->third == PF_THIRD_FFT || (l->third == PF_THIRD_CHEB && p->spec_sr && PF_CHEB_TR)) &&
                l->math == PF_PLAIN && ny % pf::p2x_tile_lines(l->precision, 1) == 0 && ny <= PF_BWD_TR_MAX_NY;
    // the forward chain on the same transposed workspace (the X pass then writes
    // rows of 16 lines at one mode); FP64 at nx = 512 only: at nx = 1024 its
    // 16-line X tile needs 136 KB of LDS (one workgroup per CU) and measured slower
    p->fwd_tr = !o.no_fwd_tr && p->bwd_tr && (l->precision == PF_F32 || nx <= 512) && PF_FWD_TR;
    if (p->share) {
        p->ws_bytes += (size_t)p->nxh * ny * nz * p->csize;
    } else if (p->blocked) {
        const size_t real_b = (size_t)nx * ny * nz * (p->csize / 2);
        const size_t cplx_b = (size_t)p->nxh * ny * nz * p->csize;
        p->ws_bytes += real_b > cplx_b ? real_b : cplx_b;
    }
    if (o.external_ws) {  // the owner supplies the workspace (pf_set_workspace)
        p->ws = nullptr;
        p->own_ws = false;
        build_passes(p);
        *out = p;
        return PF_OK;
    }
    e = hipMalloc(&p->ws, p->ws_bytes);
    if (e != hipSuccess) {
        if (p->ctl) (void)hipFree(p->ctl);
        (void)hipFree(p->tw_dev);
        delete p;
        return hip_status(e);
    }
    p->own_ws = true;
    // share-only: G starts defined (its columns beside the rank's modes are
    // transformed but never used)
    if (p->share) e = hipMemset((char *)p->ws + p->w_bytes, 0, p->ws_bytes - p->w_bytes);
    if (e != hipSuccess) {
        (void)hipFree(p->ws);
        if (p->ctl) (void)hipFree(p->ctl);
        (void)hipFree(p->tw_dev);
        delete p;
        return hip_status(e);
    }
    build_passes(p);
    *out = p;
    return PF_OK;
}

int pf_setup(int nx, int ny, int nz, const pf_layout *l, pf_plan **out) {
    return plan_create(nx, ny, nz, l, PlanOpts(), out);
}

int pf_get_dims(const pf_plan *p, int pencil, int r1, int r2, int start[3], int size[3], int order[3]) {
    if (!p) return PF_EINVAL;
    return pf_query_dims(p->nx, p->ny, p->nz, &p->lay, pencil, r1, r2, start, size, order);
}

size_t pf_workspace_bytes(const pf_plan *p) { return p ? p->ws_bytes : 0; }

int pf_set_workspace(pf_plan *p, void *ws, size_t bytes) {
    if (!p || !ws) return PF_EINVAL;
    if (((uintptr_t)ws & 255u) != 0) return PF_EALIGN;
    if (bytes < p->ws_bytes) return PF_EWORKSPACE;
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    p->ws = ws;
    p->own_ws = false;
    return PF_OK;
}

int pf_ftran_r2c(pf_plan *p, const void *in, void *out, void *stream) { return run_chain(p, 0, in, out, stream); }

int pf_btran_c2r(pf_plan *p, const void *in, void *out, void *stream) { return run_chain(p, 1, in, out, stream); }

int pf_exec_noalloc(pf_plan *p, int dir, const void *in, void *out, void *stream) {
    if (dir != PF_DIR_FORWARD && dir != PF_DIR_BACKWARD) return PF_EINVAL;
    const int rc = check_args(p, in, out);
    if (rc) return rc;
    if (p->share) return PF_EUNSUPPORTED;
    if (p->ws_bytes > kScratchBytes) return PF_EWORKSPACE;
    void *ws = scratch_address();
    if (!ws) return PF_EHIP;
    return run_chain_ws(p, dir, in, out, ws, (hipStream_t)stream, true);
}

int pf_destroy(pf_plan *p) {
    if (!p) return PF_OK;
    release_timing(p);
    for (auto &e : p->pool) {
        if (e.start) (void)hipEventDestroy(e.start);
        if (e.stop) (void)hipEventDestroy(e.stop);
    }
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    if (p->ctl) (void)hipFree(p->ctl);
    if (p->tw_dev) (void)hipFree(p->tw_dev);
    delete p;
    return PF_OK;
}

int pf_check_status(pf_plan *p) {
    if (!p) return PF_EINVAL;
    if (!p->fused || !p->ctl) return PF_OK;
    if (hipDeviceSynchronize() != hipSuccess) return PF_EHIP;
    unsigned st = 0;
    unsigned *word = p->ctl + p->fused_nq + p->nz;
    if (hipMemcpy(&st, word, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return PF_EHIP;
    if (st == 0) return PF_OK;
    if (hipMemset(word, 0, sizeof(unsigned)) != hipSuccess) return PF_EHIP;
    return PF_ETIMEOUT;
}

const char *pf_strerror(int code) {
    switch (code) {
        case PF_OK: return "ok";
        case PF_EINVAL: return "invalid argument";
        case PF_EUNSUPPORTED: return "unsupported size or option";
        case PF_EALIGN: return "pointer not aligned";
        case PF_EALIAS: return "in/out aliasing does not match the plan's in-place setting";
        case PF_ENOMEM: return "device allocation failed";
        case PF_EWORKSPACE: return "workspace missing or too small";
        case PF_EHIP: return "HIP runtime error";
        case PF_ETIMEOUT: return "a fused pass's bounded wait expired";
        default: return "unknown error";
    }
}

int pf_num_passes(const pf_plan *p, int dir) {
    if (!p || (dir != PF_DIR_FORWARD && dir != PF_DIR_BACKWARD)) return PF_EINVAL;
    return p->npass[dir];
}

int pf_run_pass(pf_plan *p, int dir, int pass, const void *in, void *out, void *stream) {
    if (!p || (dir != PF_DIR_FORWARD && dir != PF_DIR_BACKWARD)) return PF_EINVAL;
    if (pass < 0 || pass >= p->npass[dir]) return PF_EINVAL;
    if (p->share) return PF_EUNSUPPORTED;  // its passes address sub-blocks of the workspace
    if (!in || !out) return PF_EINVAL;
    if (!aligned16(in) || !aligned16(out)) return PF_EALIGN;
    return run_one(p, dir, pass, in, out, (hipStream_t)stream);
}

const char *pf_pass_name(const pf_plan *p, int dir, int pass) {
    if (!p || dir < 0 || dir > 1 || pass < 0 || pass >= p->npass[dir]) return "";
    return p->pass_names[dir][pass];
}

int pf_workspace_layout(const pf_plan *p, int dir) {
    if (!p || (dir != PF_DIR_FORWARD && dir != PF_DIR_BACKWARD)) return PF_EINVAL;
    return (dir == PF_DIR_BACKWARD && p->bwd_tr) || (dir == PF_DIR_FORWARD && p->fwd_tr) ? PF_WS_TRANSPOSED
                                                                                           : PF_WS_BLOCKED;
}

const char *pf_pass_kernel(const pf_plan *p, int dir, int pass) {
    if (!p || dir < 0 || dir > 1 || pass < 0 || pass >= p->npass[dir]) return "";
    switch (p->pass[dir][pass].kind) {
        case pf::PASS_C2C: return "c2c_generic";
        case pf::PASS_R2C_X: return "r2c_generic";
        case pf::PASS_C2R_X: return "c2r_generic";
        case pf::PASS_C2C_P2: return "c2c_pow2";
        case pf::PASS_R2C_P2: return "r2c_pow2";
        case pf::PASS_C2R_P2: return "c2r_pow2";
        case pf::PASS_C2C_MR: return "c2c_mixed";
        case pf::PASS_R2C_MR: return "r2c_mixed";
        case pf::PASS_C2R_MR: return "c2r_mixed";
        case pf::PASS_FUSED_XY: return "xy_fused";
        case pf::PASS_REMAP: return "remap";
        case pf::PASS_FILL: return "fill";
        case pf::PASS_BOX: return "box";
    }
    return "";
}

double pf_pass_bytes(const pf_plan *p, int dir, int pass) {
    if (!p || dir < 0 || dir > 1 || pass < 0 || pass >= p->npass[dir]) return 0.0;
    return p->pass_bytes[dir][pass];
}

int pf_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return PF_EINVAL;
    if (!aligned16(dst) || !aligned16(src) || (bytes & 15u)) return PF_EALIGN;
    return hip_status(pf::launch_copy(src, dst, bytes, (hipStream_t)stream));
}

int pf_probe(int kind, void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return PF_EINVAL;
    if (!aligned16(dst) || !aligned16(src) || (bytes & 15u)) return PF_EALIGN;
    hipStream_t s = (hipStream_t)stream;
    switch (kind) {
        case PF_PROBE_COPY:
            if (dst == src) return PF_EALIAS;
            return hip_status(pf::launch_copy(src, dst, bytes, s));
        case PF_PROBE_TILES:
            if (dst == src) return PF_EALIAS;
            return hip_status(pf::launch_copy_tiles(src, dst, bytes, s));
        case PF_PROBE_TILES_INPLACE:
            if (dst != src) return PF_EALIAS;
            return hip_status(pf::launch_copy_tiles(src, dst, bytes, s));
        default:
            return PF_EINVAL;
    }
}

int pf_spectral_step(pf_plan *p, const void *in, void *spec, void *out, int adjoint, void *stream) {
    if (!p || !in || !spec || !out || (adjoint != 0 && adjoint != 1)) return PF_EINVAL;
    if (p->lay.third != PF_THIRD_CHEB || p->blocked || p->share || p->lay.inplace || p->fused) return PF_EUNSUPPORTED;
    if (!aligned16(in) || !aligned16(spec) || !aligned16(out)) return PF_EALIGN;
    if (in == spec || spec == out || in == out) return PF_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    const int f64 = p->lay.precision == PF_F64;
    pf::SpecArgs a;
    a.U = spec;
    a.nx = p->nx, a.ny = p->ny, a.nz = p->nz, a.nxh = p->nxh, a.stride1 = p->lay.stride1, a.f64 = f64;
    a.conj = adjoint;
    a.scale = 1.0 / ((double)p->nx * p->ny * 2.0 * (p->nz - 1));
    if (p->spec_fused) {  // X, Y forward; Z, product, Z in one pass on W; Y, X backward
        int r = check_call(p, in, out);
        if (!r) r = run_one(p, 0, 0, in, p->ws, s);
        if (!r) r = run_one(p, 0, 1, p->ws, p->ws, s);
        if (!r) {
            pf::PassDesc d = p->spec;
            d.a.in = p->ws;
            d.a.out = p->ws;
            r = hip_status(pf::p2_spec_launch(d, adjoint, p->nx, (float)a.scale, s));
        }
        if (!r) r = run_one(p, 1, 1, p->ws, p->ws, s);
        if (!r) r = run_one(p, 1, 2, p->ws, out, s);
        return r;
    }
    const void *src = in;
    if (adjoint) {  // out = in / w(z): the adjoint of the type-I DCT is w C w^-1
        const hipError_t e = pf::launch_zweight(in, out, p->nx, p->ny, p->nz, f64, -1, s);
        if (e != hipSuccess) return hip_status(e);
        src = out;
    }
    int r = run_chain(p, 0, src, spec, stream);
    if (!r) r = hip_status(pf::launch_spec_mul(a, s));
    if (!r) r = run_chain(p, 1, spec, out, stream);
    if (!r && adjoint) r = hip_status(pf::launch_zweight(out, out, p->nx, p->ny, p->nz, f64, +1, s));
    return r;
}

int pf_set_timing(pf_plan *p, int enable) {
    if (!p) return PF_EINVAL;
    release_timing(p);
    p->timing = enable != 0;
    return PF_OK;
}

int pf_get_timing(pf_plan *p, int dir, int pass, double *total_ms, long long *count) {
    if (!p || !total_ms || !count || dir < 0 || dir > 1 || pass < 0 || pass >= p->npass[dir]) return PF_EINVAL;
    double tot = 0.0;
    long long n = 0;
    for (auto &e : p->tim[dir][pass].used) {
        if (hipEventSynchronize(e.stop) != hipSuccess) return PF_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e.start, e.stop) != hipSuccess) return PF_EHIP;
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *count = n;
    return PF_OK;
}

}  // extern "C"

struct pf_batch {
    int count = 0;
    int prec = PF_F32;
    std::vector<pf_plan *> plans;
    std::vector<size_t> roff, coff;  // byte offsets of each transform in the real / complex buffers
    size_t rbytes = 0, cbytes = 0;
    void *ws = nullptr;
    void *tables = nullptr;  // device PassArgs tables and block prefixes of the fused passes
    // fused passes: per (direction, pass) one launch per block size (threads) in the batch
    std::vector<pf::BatchLaunch> launch[2][3];
    int mode = PF_BATCH_FUSED;
    hipStream_t cap = nullptr;  // capture stream for the graph modes
    // PF_BATCH_STREAMS: the streams, the fork event (recorded on the caller's
    // stream) and one join event per stream
    hipStream_t aux[PF_BATCH_NSTREAMS] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[PF_BATCH_NSTREAMS] = {};
    std::vector<int> order;  // transforms by decreasing size
    std::vector<int> home;   // stream of each transform (serial | streams)
    struct Graph {
        const void *in = nullptr;
        void *out = nullptr;
        int mode = -1;  // the mode the launches were captured in
        hipGraphExec_t exec = nullptr;
    } graph[2];
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void batch_free(pf_batch *b) {
    if (!b) return;
    for (auto &g : b->graph)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int j = 0; j < PF_BATCH_NSTREAMS; ++j) {
        if (b->aux[j]) (void)hipStreamDestroy(b->aux[j]);
        if (b->join_ev[j]) (void)hipEventDestroy(b->join_ev[j]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    for (pf_plan *p : b->plans) pf_destroy(p);
    if (b->tables) (void)hipFree(b->tables);
    if (b->ws) (void)hipFree(b->ws);
    delete b;
}

// PF_BATCH_STREAMS: the batch's streams wait for what the caller's stream s
// has queued (fork), and s waits for everything queued on them (join).
hipError_t batch_fork(pf_batch *b, hipStream_t s) {
    hipError_t e = hipEventRecord(b->fork_ev, s);
    for (int j = 0; j < PF_BATCH_NSTREAMS && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->aux[j], b->fork_ev, 0);
    return e;
}
hipError_t batch_join(pf_batch *b, hipStream_t s) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < PF_BATCH_NSTREAMS && e == hipSuccess; ++j) {
        e = hipEventRecord(b->join_ev[j], b->aux[j]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join_ev[j], 0);
    }
    return e;
}

// Enqueue one direction of the batch on stream s in the current mode (graphs aside).
int batch_issue(pf_batch *b, int dir, const void *in, void *out, hipStream_t s) {
    const bool streams = (b->mode & PF_BATCH_STREAMS) != 0;
    if (b->mode & PF_BATCH_FUSED) {
        for (int k = 0; k < 3; ++k) {
            if (streams) {
                const hipError_t e = batch_fork(b, s);
                if (e != hipSuccess) return hip_status(e);
            }
            int j = 0;
            for (pf::BatchLaunch L : b->launch[dir][k]) {
                L.b.user_in = (const char *)in;
                L.b.user_out = (char *)out;
                // groups dealt round-robin in their order (largest blocks / lengths first)
                const hipError_t e = pf::launch_batch(L, streams ? b->aux[j] : s);
                if (e != hipSuccess) return hip_status(e);
                j = (j + 1) % PF_BATCH_NSTREAMS;
            }
            if (streams) {
                const hipError_t e = batch_join(b, s);
                if (e != hipSuccess) return hip_status(e);
            }
        }
        return PF_OK;
    }
    const bool fwd = dir == 0;
    if (streams) {
        const hipError_t e = batch_fork(b, s);
        if (e != hipSuccess) return hip_status(e);
    }
    for (int i : b->order) {
        const char *src = (const char *)in + (fwd ? b->roff[i] : b->coff[i]);
        char *dst = (char *)out + (fwd ? b->coff[i] : b->roff[i]);
        const int r = run_chain(b->plans[i], dir, src, dst, streams ? b->aux[b->home[i]] : s);
        if (r) return r;
    }
    if (streams) {
        const hipError_t e = batch_join(b, s);
        if (e != hipSuccess) return hip_status(e);
    }
    return PF_OK;
}

int batch_run(pf_batch *b, int dir, const void *in, void *out, void *stream) {
    if (!b || !in || !out) return PF_EINVAL;
    if (((uintptr_t)in & 255u) || ((uintptr_t)out & 255u)) return PF_EALIGN;
    if (in == out) return PF_EALIAS;
    hipStream_t s = (hipStream_t)stream;
    if (!(b->mode & PF_BATCH_GRAPH)) return batch_issue(b, dir, in, out, s);
    pf_batch::Graph &g = b->graph[dir];
    if (!g.exec || g.in != in || g.out != out || g.mode != b->mode) {
        if (g.exec) {  // buffers or mode changed: capture again once the old graph has finished
            if (hipStreamSynchronize(s) != hipSuccess) return PF_EHIP;
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
        }
        if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PF_EHIP;
        const int r = batch_issue(b, dir, in, out, b->cap);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &graph);
        if (r) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess) return PF_EHIP;
        const hipError_t e2 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            g.exec = nullptr;
            return PF_EHIP;
        }
        g.in = in;
        g.out = out;
        g.mode = b->mode;
    }
    return hip_status(hipGraphLaunch(g.exec, s));
}

}  // namespace

extern "C" {

int pf_batch_setup(int count, const int *dims, const pf_layout *l, const pf_tune *tune, pf_batch **out) {
    if (!out) return PF_EINVAL;
    *out = nullptr;
    if (count < 1 || !dims || !l) return PF_EINVAL;
    if (l->m1 != 1 || l->m2 != 1 || l->share_only || l->inplace || l->math != PF_PLAIN || l->fused_xy)
        return PF_EUNSUPPORTED;
    for (int i = 0; i < count; ++i) {
        const int rc = check_impl(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], l);
        if (rc) return rc;
        if (tune)
            for (int a = 0; a < 3; ++a)
                if (tune[i].radix_order[a] < 0 || tune[i].radix_order[a] > 3 || tune[i].tile[a] < 0) return PF_EINVAL;
    }
    pf_batch *b = new (std::nothrow) pf_batch();
    if (!b) return PF_ENOMEM;
    b->count = count;
    b->prec = l->precision;
    const size_t rs = l->precision == PF_F64 ? 8 : 4;
    size_t wsum = 0;
    std::vector<size_t> woff;
    for (int i = 0; i < count; ++i) {
        PlanOpts o;
        o.generic_only = true;
        o.external_ws = true;
        if (tune)
            for (int a = 0; a < 3; ++a) o.radix_order[a] = tune[i].radix_order[a], o.tile[a] = tune[i].tile[a];
        pf_plan *p = nullptr;
        const int rc = plan_create(dims[3 * i], dims[3 * i + 1], dims[3 * i + 2], l, o, &p);
        if (rc) {
            batch_free(b);
            return rc;
        }
        b->plans.push_back(p);
        woff.push_back(wsum);
        wsum += align256(p->ws_bytes);
        const size_t nr = (size_t)p->nx * p->ny * p->nz, nc = (size_t)p->nxh * p->ny * p->nz;
        b->roff.push_back(b->rbytes);
        b->coff.push_back(b->cbytes);
        b->rbytes += align256(nr * rs);
        b->cbytes += align256(nc * 2 * rs);
    }
    if (hipMalloc(&b->ws, wsum) != hipSuccess) {
        b->ws = nullptr;
        batch_free(b);
        return PF_ENOMEM;
    }
    for (int i = 0; i < count; ++i) {
        b->plans[i]->ws = (char *)b->ws + woff[i];
        b->plans[i]->own_ws = false;
    }
    // fused passes: per (direction, pass) a PassArgs table and block prefixes.
    // Transforms are grouped by block size (sorted, largest first), one launch
    // per group: a transform tuned to narrow tiles keeps its own small blocks
    // instead of running in the largest block of the batch with most lanes idle.
    const size_t tab = align256(count * sizeof(PassArgs)), pre = align256((2 * count + 1) * sizeof(long long));
    if (hipMalloc(&b->tables, 6 * (tab + pre)) != hipSuccess) {
        b->tables = nullptr;
        batch_free(b);
        return PF_ENOMEM;
    }
    std::vector<unsigned char> host(6 * (tab + pre), 0);
    std::vector<int> order(count);
    for (int dir = 0; dir < 2; ++dir)
        for (int k = 0; k < 3; ++k) {
            const size_t at = (size_t)(dir * 3 + k) * (tab + pre);
            PassArgs *A = reinterpret_cast<PassArgs *>(host.data() + at);
            long long *F = reinterpret_cast<long long *>(host.data() + at + tab);
            const PassArgs *Adev = reinterpret_cast<const PassArgs *>((char *)b->tables + at);
            const long long *Fdev = reinterpret_cast<const long long *>((char *)b->tables + at + tab);
            // user side of this pass: forward X reads / backward X writes the real
            // arrays; forward Z writes / backward Z reads the complex arrays
            const bool xpass = (dir == 0 && k == 0) || (dir == 1 && k == 2);
            const int in_user = k == 0, out_user = k == 2;
            // launch groups: runtime-radix passes by block size; compile-time
            // mixed-radix passes by length (one kernel per length)
            auto is_mr = [](pf::PassKind kd) {
                return kd == pf::PASS_C2C_MR || kd == pf::PASS_R2C_MR || kd == pf::PASS_C2R_MR;
            };
            auto mr_len = [&](int i) {
                const PassDesc &d = b->plans[i]->pass[dir][k];
                return is_mr(d.kind) ? d.a.fft.n : 0;
            };
            auto same_group = [&](int u, int v) {
                const PassDesc &du = b->plans[u]->pass[dir][k], &dv = b->plans[v]->pass[dir][k];
                return du.kind == dv.kind && mr_len(u) == mr_len(v) && du.threads == dv.threads;
            };
            for (int i = 0; i < count; ++i) {
                order[i] = i;
                const pf::PassKind kd = b->plans[i]->pass[dir][k].kind;
                if (kd != pf::PASS_C2C && kd != pf::PASS_R2C_X && kd != pf::PASS_C2R_X && !is_mr(kd)) {
                    batch_free(b);
                    return PF_EUNSUPPORTED;
                }
            }
            std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
                const PassDesc &du = b->plans[u]->pass[dir][k], &dv = b->plans[v]->pass[dir][k];
                if (du.kind != dv.kind) return du.kind < dv.kind;
                if (mr_len(u) != mr_len(v)) return mr_len(u) > mr_len(v);
                return du.threads > dv.threads;
            });
            int f = 0;  // next free prefix slot
            for (int j = 0; j < count;) {
                const int lead = order[j];
                const unsigned thr = b->plans[lead]->pass[dir][k].threads;
                pf::BatchLaunch L;
                std::memset(&L, 0, sizeof(L));
                const PassDesc &d0 = b->plans[order[j]]->pass[dir][k];
                L.kind = d0.kind;
                L.dir = d0.dir;
                L.prec = d0.prec;
                L.n = mr_len(lead);
                L.threads = thr;
                L.b.in_user = in_user;
                L.b.out_user = out_user;
                L.b.args = Adev + j;
                L.b.first = Fdev + f;
                long long blocks = 0;
                int n = 0;
                for (; j < count && same_group(order[j], lead); ++j, ++n) {
                    const int i = order[j];
                    const PassDesc &d = b->plans[i]->pass[dir][k];
                    A[j] = d.a;
                    char *w = (char *)b->plans[i]->ws;
                    const size_t uoff = xpass ? b->roff[i] : b->coff[i];
                    A[j].in = in_user ? (const void *)uoff : (const void *)w;
                    A[j].out = out_user ? (void *)uoff : (void *)w;
                    F[f + n] = blocks;
                    blocks += d.blocks;
                    L.lds = std::max(L.lds, d.lds);
                }
                F[f + n] = blocks;
                f += n + 1;
                if (blocks > 0x7fffffffLL) {
                    batch_free(b);
                    return PF_EUNSUPPORTED;
                }
                L.blocks = (unsigned)blocks;
                L.b.count = n;
                b->launch[dir][k].push_back(L);
            }
        }
    if (hipMemcpy(b->tables, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess) {
        batch_free(b);
        return PF_EHIP;
    }
    for (int j = 0; j < PF_BATCH_NSTREAMS; ++j)  // default priority, as every stream here
        if (hipStreamCreateWithFlags(&b->aux[j], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->join_ev[j], hipEventDisableTiming) != hipSuccess) {
            batch_free(b);
            return PF_EHIP;
        }
    // serial order: largest transform first, each to the stream with the fewest points so far
    b->order.resize(count);
    b->home.assign(count, 0);
    for (int i = 0; i < count; ++i) b->order[i] = i;
    auto points = [&](int i) { return (double)b->plans[i]->nx * b->plans[i]->ny * b->plans[i]->nz; };
    std::stable_sort(b->order.begin(), b->order.end(), [&](int u, int v) { return points(u) > points(v); });
    double load[PF_BATCH_NSTREAMS] = {};
    for (int i : b->order) {
        int j = 0;
        for (int q = 1; q < PF_BATCH_NSTREAMS; ++q)
            if (load[q] < load[j]) j = q;
        b->home[i] = j;
        load[j] += points(i);
    }
    *out = b;
    return PF_OK;
}

size_t pf_batch_offset(const pf_batch *b, int which, int i) {
    if (!b || i < 0 || i >= b->count || (which != 0 && which != 1)) return (size_t)-1;
    return which == 0 ? b->roff[i] : b->coff[i];
}

size_t pf_batch_bytes(const pf_batch *b, int which) {
    if (!b || (which != 0 && which != 1)) return 0;
    return which == 0 ? b->rbytes : b->cbytes;
}

int pf_batch_set_mode(pf_batch *b, int mode) {
    if (!b || mode < 0 || mode > 7) return PF_EINVAL;
    if ((mode & PF_BATCH_GRAPH) && (mode & PF_BATCH_STREAMS)) return PF_EUNSUPPORTED;
    b->mode = mode;
    return PF_OK;
}

int pf_batch_ftran_r2c(pf_batch *b, const void *in, void *out, void *stream) { return batch_run(b, 0, in, out, stream); }

int pf_batch_btran_c2r(pf_batch *b, const void *in, void *out, void *stream) { return batch_run(b, 1, in, out, stream); }

int pf_batch_destroy(pf_batch *b) {
    batch_free(b);
    return PF_OK;
}

}  // extern "C"
