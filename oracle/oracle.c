/*
 * oracle.c -- plain, slow, CPU FP64 reference for the pencil 3D R2C / C2R
 * transform of Pekurovsky, "P3DFFT: a framework for parallel computations of
 * Fourier transforms in three dimensions" (arXiv:1905.02803).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no code, header, table or constant with the HIP library: it is an
 * independent statement of what the transform computes.
 *
 * What is computed (Sec. 2, Fig. 2; Sec. 3.2, Table 1):
 *   forward  U[kz][ky][kx] = sum_{x,y,z} u[z][y][x] *
 *            exp(-2 pi i (kx x/Nx + ky y/Ny + kz z/Nz)),  kx < Nx/2+1 (integer
 *            division), all ky, kz.  The three sums are taken one axis at a
 *            time (X, then Y, then Z), as the three compute stages of the
 *            method do; the result is the 3D DFT up to rounding order.
 *   backward the staged complex-to-real transform: inverse (sign +1,
 *            unnormalised) C2C along Z, then along Y, then the 1D C2R along X
 *            of every line, which uses only Re C[0] and, for even Nx,
 *            Re C[Nx/2] (the two modes Sec. 3.2 states are real).
 *   Neither direction is normalised, so backward(forward(u)) = Nx Ny Nz u
 *   (Sec. 4.1: the round trip returns the input up to a scale factor).
 *
 * Arrays are C order, slowest index first: real u is [nz][ny][nx] (the
 * paper's Fortran "XYZ"), the half spectrum is [nz][ny][nxh] of interleaved
 * (re, im) doubles.  Layout permutations to the paper's other storage orders
 * are done by the Python wrapper (pure index permutations).
 *
 * Two 1D engines, both in FP64:
 *   (i)  direct DFT: out[k] = sum_j in[j] w^(j k mod n), O(n^2);
 *   (ii) recursive mixed-radix Cooley-Tukey decimation in time (Cooley and
 *        Tukey 1965, the algorithm the paper builds on): split by the
 *        smallest prime factor p, transform the p decimated sub-sequences,
 *        combine with twiddles by a direct p-term sum.  Any prime is handled
 *        by the same combine step, so every length is supported.
 * Twiddles are exp(sign 2 pi i r / n) with the integer r reduced mod n
 * before the libm cos/sin call, tabulated once per length.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

static const double TWO_PI = 6.28318530717958647692528676655900576839;

/* w[r] = exp(sign * 2 pi i r / n), r in [0, n) */
static cplx *roots_table(int n, int sign) {
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
    if (!w) return NULL;
    for (int r = 0; r < n; ++r) {
        double a = TWO_PI * (double)r / (double)n;
        w[r].re = cos(a);
        w[r].im = (double)sign * sin(a);
    }
    return w;
}

static int smallest_prime_factor(int n) {
    for (int p = 2; (long)p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* (i) direct DFT of one line; w is the n-th roots table of the wanted sign */
static void dft_direct(int n, const cplx *in, long istride, cplx *out, const cplx *w) {
    for (int k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < n; ++j) {
            long r = ((long)j * k) % n;
            const cplx a = in[(long)j * istride];
            sr += a.re * w[r].re - a.im * w[r].im;
            si += a.re * w[r].im + a.im * w[r].re;
        }
        out[k].re = sr;
        out[k].im = si;
    }
}

/*
 * (ii) recursive mixed-radix FFT of one line of length n read with stride
 * istride, written contiguously to out.  w is the roots table of the top
 * level length ntop (n divides ntop); scratch holds at least n entries.
 *   X[k + m s] = sum_{q<p} w_n^{q (k + m s)} Y_q[k],  Y_q = DFT_m(x[q + p j])
 */
static void fft_rec(int n, const cplx *in, long istride, cplx *out, const cplx *w, int ntop,
                    cplx *scratch) {
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_prime_factor(n);
    int m = n / p;
    for (int q = 0; q < p; ++q) fft_rec(m, in + (long)q * istride, istride * p, out + (long)q * m, w, ntop, scratch);
    long step = ntop / n; /* w_n^t = w_ntop^(t * ntop/n) */
    for (int s = 0; s < p; ++s) {
        for (int k = 0; k < m; ++k) {
            long kk = (long)k + (long)m * s;
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < p; ++q) {
                long r = (((long)q * kk) % n) * step;
                const cplx a = out[(long)q * m + k];
                sr += a.re * w[r].re - a.im * w[r].im;
                si += a.re * w[r].im + a.im * w[r].re;
            }
            scratch[kk].re = sr;
            scratch[kk].im = si;
        }
    }
    memcpy(out, scratch, sizeof(cplx) * (size_t)n);
}

/* one 1D transform with the chosen engine (0 = direct, 1 = FFT) */
static void line_transform(int engine, int n, const cplx *in, long istride, cplx *out, const cplx *w,
                           cplx *scratch) {
    if (engine == 0)
        dft_direct(n, in, istride, out, w);
    else
        fft_rec(n, in, istride, out, w, n, scratch);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int omp_thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* ---- 1D entry points (for pinning the engines) ------------------------- */

/* out[k] = sum_j in[j] exp(sign 2 pi i j k / n); in/out interleaved (re, im) */
int oracle_dft1d(int n, const double *in, double *out, int sign) {
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    cplx *w = roots_table(n, sign);
    if (!w) return -2;
    dft_direct(n, (const cplx *)in, 1, (cplx *)out, w);
    free(w);
    return 0;
}

int oracle_fft1d(int n, const double *in, double *out, int sign) {
    if (n < 1 || (sign != 1 && sign != -1)) return -1;
    cplx *w = roots_table(n, sign);
    cplx *s = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!w || !s) {
        free(w);
        free(s);
        return -2;
    }
    fft_rec(n, (const cplx *)in, 1, (cplx *)out, w, n, s);
    free(w);
    free(s);
    return 0;
}

/* ---- axis passes over a [nz][ny][nc] complex array, in place ------------ */

/* C2C along Y for every (z, c) line of A[nz][ny][nc] */
static int pass_y(int engine, int nc, int ny, int nz, cplx *A, int sign) {
    cplx *w = roots_table(ny, sign);
    if (!w) return -2;
    int err = 0;
    cplx *pool = (cplx *)malloc(sizeof(cplx) * (size_t)ny * 3 * (size_t)oracle_num_threads());
    if (!pool) err = -2;
    if (!err) {
#pragma omp parallel
    {
        cplx *a = pool + (size_t)ny * 3 * (size_t)omp_thread_id();
        cplx *b = a + ny;
        cplx *s = b + ny;
#pragma omp for schedule(static)
        for (long L = 0; L < (long)nz * nc; ++L) {
            long z = L / nc, c = L % nc;
            cplx *base = A + (z * ny) * (long)nc + c;
            for (int y = 0; y < ny; ++y) a[y] = base[(long)y * nc];
            line_transform(engine, ny, a, 1, b, w, s);
            for (int y = 0; y < ny; ++y) base[(long)y * nc] = b[y];
        }
    }
    }
    free(pool);
    free(w);
    return err;
}

/* C2C along Z for every (y, c) line of A[nz][ny][nc] */
static int pass_z(int engine, int nc, int ny, int nz, cplx *A, int sign) {
    cplx *w = roots_table(nz, sign);
    if (!w) return -2;
    int err = 0;
    long plane = (long)ny * nc;
    cplx *pool = (cplx *)malloc(sizeof(cplx) * (size_t)nz * 3 * (size_t)oracle_num_threads());
    if (!pool) err = -2;
    if (!err) {
#pragma omp parallel
    {
        cplx *a = pool + (size_t)nz * 3 * (size_t)omp_thread_id();
        cplx *b = a + nz;
        cplx *s = b + nz;
#pragma omp for schedule(static)
        for (long L = 0; L < plane; ++L) {
            cplx *base = A + L;
            for (int z = 0; z < nz; ++z) a[z] = base[(long)z * plane];
            line_transform(engine, nz, a, 1, b, w, s);
            for (int z = 0; z < nz; ++z) base[(long)z * plane] = b[z];
        }
    }
    }
    free(pool);
    free(w);
    return err;
}

/* fetch element i of a real array stored as float (is_f32) or double */
static inline double rget(const void *p, int is_f32, long i) {
    return is_f32 ? (double)((const float *)p)[i] : ((const double *)p)[i];
}
static inline cplx cget(const void *p, int is_f32, long i) {
    cplx c;
    if (is_f32) {
        c.re = (double)((const float *)p)[2 * i];
        c.im = (double)((const float *)p)[2 * i + 1];
    } else {
        c = ((const cplx *)p)[i];
    }
    return c;
}

/* ---- 3D forward: real [nz][ny][nx] -> half spectrum [nz][ny][nxh] ------ */

/* X stage: 1D real-to-complex transform of `lines` contiguous real lines of
 * length nx, keeping modes 0 .. nx/2 of each (Sec. 3.2) */
static int stage_x_r2c(int engine, int nx, long lines, const void *u, int u_is_f32, cplx *U) {
    int nxh = nx / 2 + 1;
    cplx *w = roots_table(nx, -1);
    if (!w) return -2;
    int err = 0;
    cplx *pool = (cplx *)malloc(sizeof(cplx) * (size_t)nx * 3 * (size_t)oracle_num_threads());
    if (!pool) err = -2;
    if (!err) {
#pragma omp parallel
        {
            cplx *a = pool + (size_t)nx * 3 * (size_t)omp_thread_id();
            cplx *b = a + nx;
            cplx *s = b + nx;
#pragma omp for schedule(static)
            for (long L = 0; L < lines; ++L) {
                for (int x = 0; x < nx; ++x) {
                    a[x].re = rget(u, u_is_f32, L * nx + x);
                    a[x].im = 0.0;
                }
                line_transform(engine, nx, a, 1, b, w, s);
                memcpy(U + L * nxh, b, sizeof(cplx) * (size_t)nxh);
            }
        }
    }
    free(pool);
    free(w);
    return err;
}

/*
 * Forward: the X stage, then the Y stage and the Z stage, complex-to-complex
 * (Sec. 2, Fig. 2).  engine: 0 = direct DFT per axis, 1 = recursive FFT.
 * u is float when u_is_f32, else double; U is always double.
 */
int oracle_r2c3d_ex(int engine, int nx, int ny, int nz, const void *u, int u_is_f32, double *Uout) {
    if (nx < 1 || ny < 1 || nz < 1 || (engine != 0 && engine != 1)) return -1;
    int nxh = nx / 2 + 1;
    cplx *U = (cplx *)Uout;
    int err = stage_x_r2c(engine, nx, (long)ny * nz, u, u_is_f32, U);
    if (err) return err;
    if ((err = pass_y(engine, nxh, ny, nz, U, -1))) return err;
    return pass_z(engine, nxh, ny, nz, U, -1);
}

int oracle_r2c3d(int nx, int ny, int nz, const double *u, double *U) {
    return oracle_r2c3d_ex(1, nx, ny, nz, u, 0, U);
}

/*
 * The stages on their own, for stage-level checks: the X stage of the forward
 * transform (real [nz][ny][nx] -> [nz][ny][nxh], nothing else), and one C2C
 * stage along Y (axis 1) or Z (axis 2) of a [nz][ny][nxh] array in place.
 */
int oracle_stage_x_r2c(int nx, int ny, int nz, const void *u, int u_is_f32, double *Uout) {
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    return stage_x_r2c(1, nx, (long)ny * nz, u, u_is_f32, (cplx *)Uout);
}

int oracle_stage_c2c(int nx, int ny, int nz, double *U, int axis, int sign) {
    if (nx < 1 || ny < 1 || nz < 1 || (sign != 1 && sign != -1)) return -1;
    int nxh = nx / 2 + 1;
    if (axis == 1) return pass_y(1, nxh, ny, nz, (cplx *)U, sign);
    if (axis == 2) return pass_z(1, nxh, ny, nz, (cplx *)U, sign);
    return -1;
}

/*
 * Chebyshev (cosine) third transform along z (Sec. 3.1 allows a Chebyshev
 * transform in place of the third FFT): the type-I discrete cosine transform
 * on the nz Gauss-Lobatto points, unnormalised, written out from its
 * definition,
 *   Y[k] = x[0] + (-1)^k x[nz-1] + 2 sum_{j=1}^{nz-2} x[j] cos(pi j k / (nz-1)),
 * applied to the real and imaginary parts of every z line of U[nz][ny][nxh]
 * (the matrix is real, so complex lines go through unchanged in type).  The
 * angle pi j k / (nz-1) is reduced exactly as (j k mod 2(nz-1)) / (2(nz-1)).
 */
int oracle_stage_dct1_z(int nx, int ny, int nz, double *Uio) {
    if (nx < 1 || ny < 1 || nz < 2) return -1;
    const int nxh = nx / 2 + 1;
    const long L = 2L * (nz - 1);
    double *c = (double *)malloc(sizeof(double) * (size_t)L);
    cplx *pool = (cplx *)malloc(sizeof(cplx) * (size_t)nz * 2 * (size_t)oracle_num_threads());
    if (!c || !pool) {
        free(c);
        free(pool);
        return -2;
    }
    for (long m = 0; m < L; ++m) c[m] = cos(TWO_PI * (double)m / (double)L);
    cplx *U = (cplx *)Uio;
    const long lines = (long)nxh * ny, zs = (long)nxh * ny;
#pragma omp parallel
    {
        cplx *x = pool + (size_t)nz * 2 * (size_t)omp_thread_id();
        cplx *y = x + nz;
#pragma omp for schedule(static)
        for (long ln = 0; ln < lines; ++ln) {
            for (int j = 0; j < nz; ++j) x[j] = U[ln + j * zs];
            for (int k = 0; k < nz; ++k) {
                const double sg = (k % 2 == 0) ? 1.0 : -1.0;
                double re = x[0].re + sg * x[nz - 1].re, im = x[0].im + sg * x[nz - 1].im;
                for (int j = 1; j < nz - 1; ++j) {
                    const double w = 2.0 * c[((long)j * k) % L];
                    re += w * x[j].re;
                    im += w * x[j].im;
                }
                y[k].re = re;
                y[k].im = im;
            }
            for (int k = 0; k < nz; ++k) U[ln + k * zs] = y[k];
        }
    }
    free(pool);
    free(c);
    return 0;
}

/*
 * 1D complex-to-real of one line c[0..nxh): the inverse DFT of the Hermitian
 * extension F, with F[0] = Re c[0], F[k] = c[k] and F[nx-k] = conj(c[k]) for
 * 0 < k <= (nx-1)/2, and F[nx/2] = Re c[nx/2] for even nx; out = Re(IDFT F).
 * Written out, out[x] = Re c[0] + 2 sum_k Re(c[k] e^{+2 pi i k x/nx})
 *                       + [nx even] Re c[nx/2] (-1)^x.
 */
static void c2r_line(int engine, int nx, const cplx *c, double *out, const cplx *wplus, cplx *F, cplx *G,
                     cplx *s) {
    for (int k = 0; k < nx; ++k) F[k].re = F[k].im = 0.0;
    F[0].re = c[0].re;
    int kint = (nx - 1) / 2;
    for (int k = 1; k <= kint; ++k) {
        F[k] = c[k];
        F[nx - k].re = c[k].re;
        F[nx - k].im = -c[k].im;
    }
    if (nx % 2 == 0) F[nx / 2].re = c[nx / 2].re;
    line_transform(engine, nx, F, 1, G, wplus, s);
    for (int x = 0; x < nx; ++x) out[x] = G[x].re;
}

/* X stage of the backward transform: 1D C2R of `lines` lines of nxh modes */
static int stage_x_c2r(int engine, int nx, long lines, const cplx *T, double *u) {
    int nxh = nx / 2 + 1;
    cplx *w = roots_table(nx, +1);
    if (!w) return -2;
    int err = 0;
    cplx *pool = (cplx *)malloc(sizeof(cplx) * (size_t)nx * 3 * (size_t)oracle_num_threads());
    if (!pool) err = -2;
    if (!err) {
#pragma omp parallel
        {
            cplx *F = pool + (size_t)nx * 3 * (size_t)omp_thread_id();
            cplx *G = F + nx;
            cplx *s = G + nx;
#pragma omp for schedule(static)
            for (long L = 0; L < lines; ++L) c2r_line(engine, nx, T + L * nxh, u + L * nx, w, F, G, s);
        }
    }
    free(pool);
    free(w);
    return err;
}

static cplx *promote_complex(const void *U, int U_is_f32, long M) {
    cplx *T = (cplx *)malloc(sizeof(cplx) * (size_t)M);
    if (!T) return NULL;
    for (long i = 0; i < M; ++i) T[i] = cget(U, U_is_f32, i);
    return T;
}

/* ---- 3D backward (staged): [nz][ny][nxh] -> real [nz][ny][nx] ---------- */
int oracle_c2r3d_ex(int engine, int nx, int ny, int nz, const void *Uin, int U_is_f32, double *u) {
    if (nx < 1 || ny < 1 || nz < 1 || (engine != 0 && engine != 1)) return -1;
    int nxh = nx / 2 + 1;
    long M = (long)nxh * ny * nz;
    cplx *T = promote_complex(Uin, U_is_f32, M);
    if (!T) return -2;
    int err = pass_z(engine, nxh, ny, nz, T, +1);
    if (!err) err = pass_y(engine, nxh, ny, nz, T, +1);
    if (!err) err = stage_x_c2r(engine, nx, (long)ny * nz, T, u);
    free(T);
    return err;
}

int oracle_c2r3d(int nx, int ny, int nz, const double *U, double *u) {
    return oracle_c2r3d_ex(1, nx, ny, nz, U, 0, u);
}

/* the X stage of the backward transform alone: 1D C2R of every line */
int oracle_stage_x_c2r(int nx, int ny, int nz, const void *U, int U_is_f32, double *u) {
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    long lines = (long)ny * nz;
    cplx *T = promote_complex(U, U_is_f32, lines * (nx / 2 + 1));
    if (!T) return -2;
    int err = stage_x_c2r(1, nx, lines, T, u);
    free(T);
    return err;
}

/* ---- sampled exact values, for grids too large for a whole transform ---- */

/*
 * Forward values U[kz_i][ky_i][kx] for one kx and npts (ky, kz) pairs, by the
 * separable direct sums of the definition: first the X sum of every line at
 * this kx (a [nz][ny] plane), then the Y and Z sums per point.  O(N) plus
 * O(ny nz) per point.  out holds npts interleaved complex values.
 */
int oracle_r2c_points(int nx, int ny, int nz, const void *u, int u_is_f32, int kx, int npts, const int *ky,
                      const int *kz, double *out) {
    if (nx < 1 || ny < 1 || nz < 1 || kx < 0 || kx > nx / 2) return -1;
    cplx *wx = roots_table(nx, -1), *wy = roots_table(ny, -1), *wz = roots_table(nz, -1);
    cplx *P = (cplx *)malloc(sizeof(cplx) * (size_t)ny * nz);
    if (!wx || !wy || !wz || !P) {
        free(wx);
        free(wy);
        free(wz);
        free(P);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (long L = 0; L < (long)ny * nz; ++L) {
        double sr = 0.0, si = 0.0;
        for (int x = 0; x < nx; ++x) {
            long r = ((long)kx * x) % nx;
            double v = rget(u, u_is_f32, L * nx + x);
            sr += v * wx[r].re;
            si += v * wx[r].im;
        }
        P[L].re = sr;
        P[L].im = si;
    }
    for (int i = 0; i < npts; ++i) {
        if (ky[i] < 0 || ky[i] >= ny || kz[i] < 0 || kz[i] >= nz) {
            free(wx);
            free(wy);
            free(wz);
            free(P);
            return -1;
        }
        double tr = 0.0, ti = 0.0;
#pragma omp parallel for reduction(+ : tr, ti) schedule(static)
        for (int z = 0; z < nz; ++z) {
            double yr = 0.0, yi = 0.0;
            for (int y = 0; y < ny; ++y) {
                long r = ((long)ky[i] * y) % ny;
                cplx a = P[(long)z * ny + y];
                yr += a.re * wy[r].re - a.im * wy[r].im;
                yi += a.re * wy[r].im + a.im * wy[r].re;
            }
            long rz = ((long)kz[i] * z) % nz;
            tr += yr * wz[rz].re - yi * wz[rz].im;
            ti += yr * wz[rz].im + yi * wz[rz].re;
        }
        out[2 * i] = tr;
        out[2 * i + 1] = ti;
    }
    free(wx);
    free(wy);
    free(wz);
    free(P);
    return 0;
}

/*
 * Backward output line u[z0][y0][0..nx) of the staged C2R of the half
 * spectrum U[nz][ny][nxh]: the inverse Z and Y sums evaluated at (y0, z0) for
 * every kx (direct sums, O(M)), then the 1D C2R of that line.
 */
int oracle_c2r_line(int nx, int ny, int nz, const void *U, int U_is_f32, int y0, int z0, double *out) {
    if (nx < 1 || ny < 1 || nz < 1 || y0 < 0 || y0 >= ny || z0 < 0 || z0 >= nz) return -1;
    int nxh = nx / 2 + 1;
    cplx *wy = roots_table(ny, +1), *wz = roots_table(nz, +1), *wx = roots_table(nx, +1);
    cplx *c = (cplx *)malloc(sizeof(cplx) * (size_t)nxh);
    cplx *F = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    cplx *G = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    cplx *s = (cplx *)malloc(sizeof(cplx) * (size_t)nx);
    int err = 0;
    if (!wy || !wz || !wx || !c || !F || !G || !s) {
        err = -2;
        goto done;
    }
#pragma omp parallel for schedule(static)
    for (int kx = 0; kx < nxh; ++kx) {
        double tr = 0.0, ti = 0.0;
        for (int kz = 0; kz < nz; ++kz) {
            double yr = 0.0, yi = 0.0;
            for (int ky = 0; ky < ny; ++ky) {
                long r = ((long)ky * y0) % ny;
                cplx a = cget(U, U_is_f32, ((long)kz * ny + ky) * nxh + kx);
                yr += a.re * wy[r].re - a.im * wy[r].im;
                yi += a.re * wy[r].im + a.im * wy[r].re;
            }
            long rz = ((long)kz * z0) % nz;
            tr += yr * wz[rz].re - yi * wz[rz].im;
            ti += yr * wz[rz].im + yi * wz[rz].re;
        }
        c[kx].re = tr;
        c[kx].im = ti;
    }
    c2r_line(1, nx, c, out, wx, F, G, s);
done:
    free(wy);
    free(wz);
    free(wx);
    free(c);
    free(F);
    free(G);
    free(s);
    return err;
}
