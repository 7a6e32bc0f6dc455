// asan_planner.cpp -- host-only exercise of the library's planner paths, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code of
// capi.hip (tests/test_sanitizers.py).  Nothing here reaches a HIP call: every
// pf_setup / pf_batch_setup below fails validation first, and the other calls
// get NULL handles.  Besides the sanitizers' own checks it asserts that the
// Table 1 blocks of every accepted grid tile each axis exactly (the balanced
// split of uneven extents, Sec. 3.4) and that every rank's block is non-empty
// (Eq. 2 read as in pf_check).
#include <cstdio>
#include <cstdlib>
#include <initializer_list>

#include "pencilfft.h"

static int failures = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

// Blocks of one pencil over all ranks: along each axis the blocks of ranks
// sharing the other split index tile [0, n) in rank order.
static void check_tiling(int nx, int ny, int nz, const pf_layout &l, int pencil) {
    const int nxh = nx / 2 + 1;
    const int ext[3] = {pencil == PF_PENCIL_X ? nx : nxh, ny, nz};
    for (int axis = 0; axis < 3; ++axis) {
        // which split index moves this axis: X-pencil y by r1, z by r2; Y-pencil x by r1, z by r2;
        // Z-pencil x by r1, y by r2
        int by = -1;
        if (pencil == PF_PENCIL_X) by = axis == 1 ? 1 : axis == 2 ? 2 : 0;
        if (pencil == PF_PENCIL_Y) by = axis == 0 ? 1 : axis == 2 ? 2 : 0;
        if (pencil == PF_PENCIL_Z) by = axis == 0 ? 1 : axis == 1 ? 2 : 0;
        const int M = by == 1 ? l.m1 : by == 2 ? l.m2 : 1;
        int next = 0;
        for (int r = 0; r < M; ++r) {
            int start[3], size[3], order[3];
            const int r1 = by == 1 ? r : 0, r2 = by == 2 ? r : 0;
            const int rc = pf_query_dims(nx, ny, nz, &l, pencil, r1, r2, start, size, order);
            CHECK(rc == PF_OK);
            if (rc) return;
            CHECK(start[axis] == next);
            CHECK(size[axis] >= 1);
            next = start[axis] + size[axis];
            int seen = 0;
            for (int i = 0; i < 3; ++i) {
                CHECK(order[i] >= 0 && order[i] < 3);
                if (order[i] >= 0 && order[i] < 3) seen |= 1 << order[i];
            }
            CHECK(seen == 7);
        }
        CHECK(next == ext[axis]);
    }
}

int main() {
    pf_layout l;
    pf_layout_init(&l);
    CHECK(l.m1 == 1 && l.m2 == 1 && l.stride1 == 1 && l.precision == PF_F32);
    pf_layout_init(nullptr);
    for (int c = -12; c <= 3; ++c) CHECK(pf_strerror(c) != nullptr);

    static const int lens[] = {-1, 0, 1, 2, 3, 4, 5, 6, 7, 11, 13, 15, 16, 17, 48, 49, 250, 360, 480,
                               1024, 4096, 8192, 8193, 9000, 1 << 20};
    static const int grids[] = {-1, 0, 1, 2, 3, 5, 8, 1000};
    long long accepted = 0, calls = 0;
    int start[3], size[3], order[3];
    for (int nx : lens)
        for (int ny : {1, 6, 7, 13, 64, 8192, 9000})
            for (int nz : {0, 1, 2, 5, 17, 250, 8193})
                for (int m1 : grids)
                    for (int m2 : grids)
                        for (int variant = 0; variant < 6; ++variant) {
                            pf_layout_init(&l);
                            l.m1 = m1;
                            l.m2 = m2;
                            l.stride1 = variant & 1;
                            l.precision = (variant >> 1) & 1;
                            l.third = variant >= 4 ? (variant == 4 ? PF_THIRD_CHEB : PF_THIRD_EMPTY) : PF_THIRD_FFT;
                            const int rc = pf_check(nx, ny, nz, &l);
                            ++calls;
                            CHECK(rc == PF_OK || rc == PF_EINVAL || rc == PF_EUNSUPPORTED);
                            for (int pencil = -1; pencil <= 3; ++pencil)
                                for (int r1 : {-1, 0, m1 - 1, m1})
                                    for (int r2 : {-1, 0, m2 - 1, m2}) {
                                        const int q = pf_query_dims(nx, ny, nz, &l, pencil, r1, r2, start, size, order);
                                        const bool in = pencil >= 0 && pencil <= 2 && r1 >= 0 && r1 < m1 && r2 >= 0 &&
                                                        r2 < m2;
                                        CHECK(rc != PF_OK ? q == rc : (in ? q == PF_OK : q == PF_EINVAL));
                                    }
                            CHECK(pf_query_dims(nx, ny, nz, &l, PF_PENCIL_X, 0, 0, nullptr, size, order) ==
                                  (rc ? rc : PF_EINVAL));
                            if (rc == PF_OK) {
                                ++accepted;
                                for (int pencil = 0; pencil < 3; ++pencil) check_tiling(nx, ny, nz, l, pencil);
                            } else {
                                // rejected grids never reach a HIP call
                                pf_plan *p = reinterpret_cast<pf_plan *>(&l);
                                CHECK(pf_setup(nx, ny, nz, &l, &p) == rc);
                                CHECK(p == nullptr);
                            }
                        }
    // option values outside their ranges
    const int bad_fields = 12;
    for (int f = 0; f < bad_fields; ++f)
        for (int i = 0; i < 3; ++i) {
            // fields in declaration order: m1, m2, stride1, useeven, precision, math, inplace,
            // third, share_only, r1, r2, fused_xy (r1 / r2 must be 0 without share_only)
            const int grid_bad[3] = {-3, 0, 100}, enum3_bad[3] = {-3, 3, 7}, flag_bad[3] = {-3, 2, 7};
            const int v = f < 2 ? grid_bad[i] : (f == 5 || f == 7) ? enum3_bad[i] : flag_bad[i];
            pf_layout_init(&l);
            int *field = &l.m1 + f;
            *field = v;
            const int rc = pf_check(16, 16, 16, &l);
            CHECK(rc == PF_EINVAL);
            pf_plan *p = nullptr;
            CHECK(pf_setup(16, 16, 16, &l, &p) == PF_EINVAL && p == nullptr);
        }
    CHECK(pf_check(16, 16, 16, nullptr) == PF_EINVAL);
    CHECK(pf_setup(16, 16, 16, &l, nullptr) == PF_EINVAL);
    // matrix-core math with FP64 and share-only with in-place are refused before any allocation
    pf_layout_init(&l);
    l.precision = PF_F64;
    l.math = PF_MFMA_BF16X2;
    pf_plan *p = nullptr;
    CHECK(pf_setup(32, 32, 32, &l, &p) == PF_EUNSUPPORTED && p == nullptr);
    pf_layout_init(&l);
    l.share_only = 1;
    l.inplace = 1;
    CHECK(pf_setup(32, 32, 32, &l, &p) == PF_EUNSUPPORTED && p == nullptr);

    // batch validation
    pf_layout_init(&l);
    pf_batch *b = nullptr;
    const int dims[6] = {16, 8, 8, 11, 8, 8};
    CHECK(pf_batch_setup(0, dims, &l, nullptr, &b) == PF_EINVAL && b == nullptr);
    CHECK(pf_batch_setup(2, nullptr, &l, nullptr, &b) == PF_EINVAL);
    CHECK(pf_batch_setup(2, dims, nullptr, nullptr, &b) == PF_EINVAL);
    CHECK(pf_batch_setup(2, dims, &l, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_batch_setup(2, dims, &l, nullptr, &b) == PF_EUNSUPPORTED && b == nullptr);  // 11 = prime
    pf_tune tune[2] = {};
    tune[1].radix_order[2] = 9;
    const int dims2[6] = {16, 8, 8, 12, 8, 8};
    CHECK(pf_batch_setup(2, dims2, &l, tune, &b) == PF_EINVAL && b == nullptr);
    l.inplace = 1;
    CHECK(pf_batch_setup(2, dims2, &l, nullptr, &b) == PF_EUNSUPPORTED);

    // NULL handles
    CHECK(pf_get_dims(nullptr, 0, 0, 0, start, size, order) == PF_EINVAL);
    CHECK(pf_workspace_bytes(nullptr) == 0);
    CHECK(pf_set_workspace(nullptr, nullptr, 0) == PF_EINVAL);
    CHECK(pf_ftran_r2c(nullptr, nullptr, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_btran_c2r(nullptr, nullptr, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_destroy(nullptr) == PF_OK);
    CHECK(pf_num_passes(nullptr, 0) == PF_EINVAL);
    CHECK(pf_run_pass(nullptr, 0, 0, nullptr, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_pass_name(nullptr, 0, 0) != nullptr);
    CHECK(pf_pass_kernel(nullptr, 0, 0) != nullptr && pf_pass_kernel(nullptr, 0, 0)[0] == 0);
    CHECK(pf_workspace_layout(nullptr, PF_DIR_BACKWARD) == PF_EINVAL);
    CHECK(pf_pass_bytes(nullptr, 0, 0) == 0.0);
    CHECK(pf_set_timing(nullptr, 1) == PF_EINVAL);
    double ms;
    long long cnt;
    CHECK(pf_get_timing(nullptr, 0, 0, &ms, &cnt) == PF_EINVAL);
    CHECK(pf_copy(nullptr, nullptr, 16, nullptr) == PF_EINVAL);
    CHECK(pf_spectral_step(nullptr, nullptr, nullptr, nullptr, 0, nullptr) == PF_EINVAL);
    CHECK(pf_batch_offset(nullptr, 0, 0) == (size_t)-1);
    CHECK(pf_batch_bytes(nullptr, 0) == 0);
    CHECK(pf_batch_set_mode(nullptr, 0) == PF_EINVAL);
    CHECK(pf_batch_ftran_r2c(nullptr, nullptr, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_batch_btran_c2r(nullptr, nullptr, nullptr, nullptr) == PF_EINVAL);
    CHECK(pf_batch_destroy(nullptr) == PF_OK);

    std::printf("planner checks: %lld layouts, %lld accepted, %d failures\n", calls, accepted, failures);
    return failures ? 1 : 0;
}
