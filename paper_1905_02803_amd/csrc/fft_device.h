// fft_device.h -- device-side building blocks shared by the transform
// kernels: interleaved complex helpers and in-register DFTs of radix 2, 3, 4,
// 5, 7, 8 and 16 with sign DIR (-1 forward, +1 backward):
//     X[k] = sum_r x[r] exp(DIR 2 pi i r k / R).
#pragma once

#include <hip/hip_runtime.h>

namespace pf {

template <typename T>
struct V2;
template <>
struct V2<float> {
    typedef float2 t;
};
template <>
struct V2<double> {
    typedef double2 t;
};
template <typename T>
using cx = typename V2<T>::t;

template <typename T>
__device__ __forceinline__ cx<T> cmk(T a, T b) {
    cx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename V>
__device__ __forceinline__ V cadd(V a, V b) {
    V r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename V>
__device__ __forceinline__ V csub(V a, V b) {
    V r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename V, typename S>
__device__ __forceinline__ V cscale(V a, S s) {
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
// a * (DIR i)
template <int DIR, typename V>
__device__ __forceinline__ V cmuli(V a) {
    V r;
    if (DIR > 0) {
        r.x = -a.y;
        r.y = a.x;
    } else {
        r.x = a.y;
        r.y = -a.x;
    }
    return r;
}
// a * (c + DIR i s)
template <int DIR, typename V, typename S>
__device__ __forceinline__ V crot(V a, S c, S s) {
    const S sd = DIR > 0 ? s : -s;
    V r;
    r.x = a.x * c - a.y * sd;
    r.y = a.x * sd + a.y * c;
    return r;
}

// cos and sin of 2 pi m / R for the odd radices, m in [0, R).  Values of the
// closed forms (e.g. cos(2 pi/5) = (sqrt 5 - 1)/4), to 25 digits.
__device__ constexpr double odd_cos(int R, int m) {
    return R == 3 ? (m == 0 ? 1.0 : -0.5)
         : R == 5 ? (m == 0 ? 1.0 : (m == 1 || m == 4) ? 0.3090169943749474241022934 : -0.8090169943749474241022934)
         : (m == 0 ? 1.0
                   : (m == 1 || m == 6) ? 0.6234898018587335305250049
                   : (m == 2 || m == 5) ? -0.2225209339563144042889026
                                        : -0.9009688679024191262361023);
}
__device__ constexpr double odd_sin(int R, int m) {
    return R == 3 ? (m == 0 ? 0.0 : m == 1 ? 0.8660254037844386467637232 : -0.8660254037844386467637232)
         : R == 5 ? (m == 0 ? 0.0
                     : m == 1 ? 0.9510565162951535721164393
                     : m == 2 ? 0.5877852522924731291687060
                     : m == 3 ? -0.5877852522924731291687060
                              : -0.9510565162951535721164393)
         : (m == 0 ? 0.0
                   : m == 1 ? 0.7818314824680298087084445
                   : m == 2 ? 0.9749279121818236070181317
                   : m == 3 ? 0.4338837391175581204757683
                   : m == 4 ? -0.4338837391175581204757683
                   : m == 5 ? -0.9749279121818236070181317
                            : -0.7818314824680298087084445);
}

constexpr double kSqrtHalf = 0.7071067811865475244008444;   // cos(pi/4)
constexpr double kCosPi8 = 0.9238795325112867561281832;     // cos(pi/8)
constexpr double kSinPi8 = 0.3826834323650897717284600;     // sin(pi/8)

// ---- in-register DFTs of size R with sign DIR:  X[k] = sum_r x[r] e^{DIR 2 pi i r k / R}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(cx<T> &x0, cx<T> &x1, cx<T> &x2, cx<T> &x3) {
    const cx<T> t0 = cadd(x0, x2), t1 = csub(x0, x2), t2 = cadd(x1, x3);
    const cx<T> t3 = cmuli<DIR>(csub(x1, x3));
    x0 = cadd(t0, t2);
    x2 = csub(t0, t2);
    x1 = cadd(t1, t3);
    x3 = csub(t1, t3);
}

template <typename T, int R, int DIR>
struct Dft;

template <typename T, int DIR>
struct Dft<T, 2, DIR> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        const cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T, int DIR>
struct Dft<T, 4, DIR> {
    __device__ __forceinline__ static void run(cx<T> *v) { dft4<T, DIR>(v[0], v[1], v[2], v[3]); }
};

// radix 8: two radix-4 DFTs on the even and odd samples, combined with W8^k.
template <typename T, int DIR>
struct Dft<T, 8, DIR> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<T, DIR>(e0, e1, e2, e3);
        dft4<T, DIR>(o0, o1, o2, o3);
        const T c = T(kSqrtHalf);
        o1 = crot<DIR>(o1, c, c);
        o2 = cmuli<DIR>(o2);
        o3 = crot<DIR>(o3, -c, c);
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3);
        v[7] = csub(e3, o3);
    }
};

// radix 16 as 4 x 4: DFT4 over n2 of x[4 n2 + n1], twiddle W16^{n1 k1},
// DFT4 over n1; output k1 + 4 k2.
template <typename T, int DIR>
struct Dft<T, 16, DIR> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        cx<T> a[4][4];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            a[n1][0] = v[n1];
            a[n1][1] = v[n1 + 4];
            a[n1][2] = v[n1 + 8];
            a[n1][3] = v[n1 + 12];
            dft4<T, DIR>(a[n1][0], a[n1][1], a[n1][2], a[n1][3]);
        }
        const T c1 = T(kCosPi8), s1 = T(kSinPi8), h = T(kSqrtHalf);
        a[1][1] = crot<DIR>(a[1][1], c1, s1);   // W^1
        a[1][2] = crot<DIR>(a[1][2], h, h);     // W^2
        a[1][3] = crot<DIR>(a[1][3], s1, c1);   // W^3
        a[2][1] = crot<DIR>(a[2][1], h, h);     // W^2
        a[2][2] = cmuli<DIR>(a[2][2]);          // W^4
        a[2][3] = crot<DIR>(a[2][3], -h, h);    // W^6
        a[3][1] = crot<DIR>(a[3][1], s1, c1);   // W^3
        a[3][2] = crot<DIR>(a[3][2], -h, h);    // W^6
        a[3][3] = crot<DIR>(a[3][3], -c1, -s1); // W^9
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            dft4<T, DIR>(a[0][k1], a[1][k1], a[2][k1], a[3][k1]);
            v[k1] = a[0][k1];
            v[k1 + 4] = a[1][k1];
            v[k1 + 8] = a[2][k1];
            v[k1 + 12] = a[3][k1];
        }
    }
};

// odd prime radix: pair x[r] with x[R-r]; X[k] = x0 + sum s_r cos + DIR i sum d_r sin.
template <typename T, int R, int DIR>
struct DftOdd {
    __device__ __forceinline__ static void run(cx<T> *v) {
        constexpr int H = (R - 1) / 2;
        cx<T> s[H], d[H];
        cx<T> x0 = v[0], sum = v[0];
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            s[r - 1] = cadd(v[r], v[R - r]);
            d[r - 1] = csub(v[r], v[R - r]);
            sum = cadd(sum, s[r - 1]);
        }
        v[0] = sum;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            cx<T> A = x0, Bv = cmk<T>(T(0), T(0));
#pragma unroll
            for (int r = 1; r <= H; ++r) {
                const int m = (r * k) % R;
                A = cadd(A, cscale(s[r - 1], T(odd_cos(R, m))));
                Bv = cadd(Bv, cscale(d[r - 1], T(odd_sin(R, m))));
            }
            const cx<T> iB = cmuli<DIR>(Bv);
            v[k] = cadd(A, iB);
            v[R - k] = csub(A, iB);
        }
    }
};
template <typename T, int DIR>
struct Dft<T, 3, DIR> : DftOdd<T, 3, DIR> {};
template <typename T, int DIR>
struct Dft<T, 5, DIR> : DftOdd<T, 5, DIR> {};
template <typename T, int DIR>
struct Dft<T, 7, DIR> : DftOdd<T, 7, DIR> {};

}  // namespace pf
