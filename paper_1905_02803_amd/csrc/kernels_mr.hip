// kernels_mr.hip -- host side of the compile-time mixed-radix passes
// (kernels_mr.h): which lengths have them, their launch shapes, launches.
#include <cstring>

#include "kernels_mr.h"

namespace pf {

namespace {

bool mr_factors(int n, int *n1, int *n2) {
#define PF_MR_CASE(N, N1, N2) \
    case N:                   \
        *n1 = N1;             \
        *n2 = N2;             \
        return true;
    switch (n) {
        PF_MR_LENGTHS(PF_MR_CASE)
        default:
            return false;
    }
#undef PF_MR_CASE
}

const void *mr_kernel(int n, int what) {
    for (auto pick : {mr_kernel_p0, mr_kernel_p1, mr_kernel_p2, mr_kernel_p3})
        if (const void *k = pick(n, what)) return k;
    return nullptr;
}

// kernel of pass kind `kind`, direction dir (-1 forward, +1 backward)
const void *mr_kernel_for(int kind, int dir, int n) {
    const int what = kind == PASS_C2C_MR ? (dir < 0 ? 0 : 1) : kind == PASS_R2C_MR ? 2 : kind == PASS_C2R_MR ? 3 : -1;
    return what < 0 ? nullptr : mr_kernel(n, what);
}

hipError_t mr_go(const void *k, unsigned blocks, unsigned threads, size_t lds, MrArgs &m, hipStream_t s) {
    if (!k) return hipErrorInvalidValue;
    if (blocks == 0) return hipSuccess;
    void *args[] = {&m};
    return hipLaunchKernel(k, dim3(blocks), dim3(threads), args, lds, s);
}

}  // namespace

bool mr_supported(int n, int prec) {
    int a, b;
    return prec == 0 && mr_factors(n, &a, &b);
}

int mr_threads_of(int n, int xpass) {
    int a = 0, b = 0;
    if (!mr_factors(n, &a, &b)) return 0;
    return xpass ? mr_x_threads(a, b) : mr_c2c_threads(a, b);
}

int mr_x_pairs() { return PF_MR_XP; }

size_t mr_lds_bytes(int n, int xpass) {
    // the kernels' own tile constants, so that host and device sizes agree
#define PF_MR_CASE(N, N1, N2) \
    case N:                   \
        return (size_t)(xpass ? MrShape<N1, N2>::XLDS : MrShape<N1, N2>::CLDS) * sizeof(float2);
    switch (n) {
        PF_MR_LENGTHS(PF_MR_CASE)
        default:
            return 0;
    }
#undef PF_MR_CASE
}

hipError_t mr_launch(const PassDesc &d, hipStream_t s) {
    MrArgs m;
    std::memset(&m, 0, sizeof(m));
    m.one = d.a;
    return mr_go(mr_kernel_for(d.kind, d.dir, d.a.fft.n), d.blocks, d.threads, d.lds, m, s);
}

hipError_t mr_launch_batch(const BatchLaunch &L, hipStream_t s) {
    MrArgs m;
    std::memset(&m, 0, sizeof(m));
    m.b = L.b;
    if (m.b.count < 1) return hipErrorInvalidValue;
    return mr_go(mr_kernel_for(L.kind, L.dir, L.n), L.blocks, L.threads, L.lds, m, s);
}

}  // namespace pf
