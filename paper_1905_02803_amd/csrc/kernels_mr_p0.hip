// kernels_mr_p0.hip -- the compile-time mixed-radix kernels of the lengths in
// PF_MR_LENGTHS_0 (one of four units, built in parallel).
#include "kernels_mr.h"

namespace pf {

const void *mr_kernel_p0(int n, int what) {
#define PF_MR_CASE(N, N1, N2) \
    case N:                   \
        return mr_kernel_of<N1, N2>(what);
    switch (n) {
        PF_MR_LENGTHS_0(PF_MR_CASE)
        default:
            return nullptr;
    }
#undef PF_MR_CASE
}

}  // namespace pf
