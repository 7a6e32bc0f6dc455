// fused_schedule.h -- the work order of the fused X-Y pass (k_xy_fused), shared
// by the kernel and the host-side schedule test.
//
// A queue holds the planes q, q + nq, q + 2 nq, ... (np of them, positions
// j = 0 .. np-1).  Each plane has pi producer items (the stage that runs
// first) and ci consumer items (the stage that needs all of the plane's
// producer output).  The queue's items are ordered
//     P(0) .. P(L-1), then P(j+L), C(j) for j = 0 .. np-L-1, then C(np-L) .. C(np-1)
// with L = min(lag, np): producers run L planes ahead of consumers, and every
// consumer item comes after all producer items of its plane.
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

// Item k of a queue: kind (0 producer, 1 consumer), the plane's position j
// in the queue and the item's index within the plane; false past the end
// (np (pi + ci) items).
__host__ __device__ inline bool fused_item(int k, int np, int lag, int pi, int ci, int &kind, int &j, int &idx) {
    if (k < 0) return false;
    const int L = lag < np ? lag : np;
    if (k < L * pi) {
        kind = 0, j = k / pi, idx = k - j * pi;
        return true;
    }
    k -= L * pi;
    const int nfull = np - L, g = pi + ci;
    if (k < nfull * g) {
        const int jj = k / g, r = k - jj * g;
        if (r < pi) kind = 0, j = jj + L, idx = r;
        else kind = 1, j = jj, idx = r - pi;
        return true;
    }
    k -= nfull * g;
    if (k >= L * ci) return false;
    kind = 1, j = nfull + k / ci, idx = k - (k / ci) * ci;
    return true;
}

}  // namespace pf
