// HIP kernels for gfx950: the double-grid Ga operator (Algorithm 2) as
// fused FFT passes, conjugate-gradient vector kernels, FP64 energy quadrature,
// and the material setup (eq. MBA_GA, eq. inclcomp_formula, Lemma grid_compos).
//
// Transforms are mixed-radix (3, 5, 7) self-sorting Stockham DFTs staged in
// LDS; every grid size is odd (M >= 2N-1 odd and 3,5,7-smooth), so no radix 2
// and no Nyquist frequency ever occurs.
#include "fftgal_internal.h"

#include <type_traits>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace fftgal {
namespace {

template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = float2; };
template <> struct VecOf<double> { using type = double2; };

template <typename T> using Vt = typename VecOf<T>::type;

// The argument tables hold generic pointers; operands known to live in device
// global memory are cast to that address space so that the compiler emits
// global (not flat) accesses and may move them past LDS accesses.
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T *gbl(T *p) {
    return (__attribute__((address_space(1))) T *)(p);
}

template <typename T>
__device__ __forceinline__ Vt<T> mk(T a, T b) {
    Vt<T> v;
    v.x = a;
    v.y = b;
    return v;
}
// complex loads and stores through global-address-space pointers, as one
// 8- or 16-byte access of a native two-element vector
template <typename V> struct ScalarOf;
template <> struct ScalarOf<float2> { using type = float; };
template <> struct ScalarOf<double2> { using type = double; };
template <typename S> using NVec2 = S __attribute__((ext_vector_type(2)));
template <typename V> __device__ __forceinline__ V gld(const __attribute__((address_space(1))) V *p) {
    using S = typename ScalarOf<V>::type;
    const NVec2<S> w = *reinterpret_cast<const __attribute__((address_space(1))) NVec2<S> *>(p);
    V v;
    v.x = w.x;
    v.y = w.y;
    return v;
}
template <typename V> __device__ __forceinline__ void gst(__attribute__((address_space(1))) V *p, V v) {
    using S = typename ScalarOf<V>::type;
    NVec2<S> w;
    w.x = v.x;
    w.y = v.y;
    *reinterpret_cast<__attribute__((address_space(1))) NVec2<S> *>(p) = w;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <typename V> __device__ __forceinline__ V csub(V a, V b) {
    a.x -= b.x;
    a.y -= b.y;
    return a;
}
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// cos(2 pi j / R) and sin(2 pi j / R), 0 <= j <= (R - 1) / 2.
template <int R> __device__ constexpr double ccos(int j);
template <int R> __device__ constexpr double csin(int j);
template <> __device__ constexpr double ccos<3>(int j) { return j == 0 ? 1.0 : -0.5; }
template <> __device__ constexpr double csin<3>(int j) {
    return j == 0 ? 0.0 : 0.86602540378443864676372317075294;
}
template <> __device__ constexpr double ccos<5>(int j) {
    return j == 0 ? 1.0 : j == 1 ? 0.30901699437494742410229341718282 : -0.80901699437494742410229341718282;
}
template <> __device__ constexpr double csin<5>(int j) {
    return j == 0 ? 0.0 : j == 1 ? 0.95105651629515357211643933337938 : 0.58778525229247312916870595463907;
}
template <> __device__ constexpr double ccos<7>(int j) {
    return j == 0 ? 1.0
         : j == 1 ? 0.62348980185873353052500488400424
         : j == 2 ? -0.22252093395631440428890256449680
                  : -0.90096886790241912623610231950745;
}
template <> __device__ constexpr double csin<7>(int j) {
    return j == 0 ? 0.0
         : j == 1 ? 0.78183148246802980870844452667406
         : j == 2 ? 0.97492791218182360701813168299393
                  : 0.43388373911755812047576833284836;
}

// In-register DFT of odd length R: U[m] = sum_q u[q] exp(sg 2 pi i q m / R),
// computed from the symmetric and antisymmetric pair sums u[q] +- u[R-q].
template <typename T, int R>
__device__ __forceinline__ void dft(Vt<T> *u, T sg) {
    constexpr int H = (R - 1) / 2;
    Vt<T> sp[H], sm[H];
#pragma unroll
    for (int q = 1; q <= H; ++q) {
        sp[q - 1] = cadd(u[q], u[R - q]);
        sm[q - 1] = csub(u[q], u[R - q]);
    }
    const Vt<T> u0 = u[0];
    Vt<T> tot = u0;
#pragma unroll
    for (int q = 0; q < H; ++q) tot = cadd(tot, sp[q]);
#pragma unroll
    for (int m = 1; m <= H; ++m) {
        Vt<T> a = u0;
        Vt<T> b = mk<T>(T(0), T(0));
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            const int j = (q * m) % R;
            const T cv = T(j <= H ? ccos<R>(j) : ccos<R>(R - j));
            const T sv = T(j <= H ? csin<R>(j) : -csin<R>(R - j));
            a.x += cv * sp[q - 1].x;
            a.y += cv * sp[q - 1].y;
            b.x += sv * sm[q - 1].x;
            b.y += sv * sm[q - 1].y;
        }
        b.x *= sg;
        b.y *= sg;
        u[m] = mk<T>(a.x - b.y, a.y + b.x);
        u[R - m] = mk<T>(a.x + b.y, a.y - b.x);
    }
    u[0] = tot;
}

constexpr double kPiD = 3.14159265358979323846;
constexpr double cx_sin_small(double x) {
    double x2 = x * x, t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x2 / ((2.0 * k) * (2.0 * k + 1.0));
        s += t;
    }
    return s;
}
constexpr double cx_cos_small(double x) {
    double x2 = x * x, t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
        s += t;
    }
    return s;
}
// cos and sin of 2 pi j / R by exact quadrant reduction of the rational j/R
// and Taylor series on [0, pi/4] (evaluated at compile time).
template <int R> struct TrigTab {
    double c[R], s[R];
    constexpr TrigTab() : c(), s() {
        for (int j = 0; j < R; ++j) {
            const int q = (4 * j) / R, r = 4 * j - q * R;
            double cc = 0.0, ss = 0.0;
            if (2 * r <= R) {
                const double t = (kPiD / 2) * r / R;
                cc = cx_cos_small(t);
                ss = cx_sin_small(t);
            } else {
                const double u = (kPiD / 2) * (R - r) / R;
                cc = cx_sin_small(u);
                ss = cx_cos_small(u);
            }
            c[j] = q == 0 ? cc : q == 1 ? -ss : q == 2 ? -cc : ss;
            s[j] = q == 0 ? ss : q == 1 ? cc : q == 2 ? -ss : -cc;
        }
    }
};
template <int R> struct Trig { static constexpr TrigTab<R> v{}; };

constexpr int smallest_prime_factor(int n) {
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

// In-register DFT of length R (any product of 3, 5, 7): prime lengths use the
// symmetric butterflies above, composite ones R = R1 R2 a Cooley-Tukey split
// (R2 DFTs of length R1, twiddles exp(sg 2 pi i n2 k1 / R), R1 DFTs of length
// R2, output index k1 + R1 k2).
template <typename T, int R>
__device__ __forceinline__ void dftn(Vt<T> *u, T sg) {
    if constexpr (R == 3 || R == 5 || R == 7) {
        dft<T, R>(u, sg);
    } else if constexpr (R == 15) {
        // Good-Thomas split 15 = 3 * 5 (coprime, no twiddles): input index
        // (5 n1 + 3 n2) mod 15, output index (10 k1 + 6 k2) mod 15
        Vt<T> y[3][5];
#pragma unroll
        for (int n2 = 0; n2 < 5; ++n2) {
            Vt<T> col[3];
#pragma unroll
            for (int n1 = 0; n1 < 3; ++n1) col[n1] = u[(5 * n1 + 3 * n2) % 15];
            dft<T, 3>(col, sg);
#pragma unroll
            for (int k1 = 0; k1 < 3; ++k1) y[k1][n2] = col[k1];
        }
#pragma unroll
        for (int k1 = 0; k1 < 3; ++k1) {
            dft<T, 5>(y[k1], sg);
#pragma unroll
            for (int k2 = 0; k2 < 5; ++k2) u[(10 * k1 + 6 * k2) % 15] = y[k1][k2];
        }
    } else {
        constexpr int R1 = smallest_prime_factor(R);
        constexpr int R2 = R / R1;
        Vt<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
            Vt<T> col[R1];
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) col[n1] = u[n1 * R2 + n2];
            dftn<T, R1>(col, sg);
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                const int j = (n2 * k1) % R;
                if (j == 0) {
                    y[k1 * R2 + n2] = col[k1];
                } else {
                    const T c = T(Trig<R>::v.c[j]);
                    const T sn = sg * T(Trig<R>::v.s[j]);
                    y[k1 * R2 + n2] = mk<T>(col[k1].x * c - col[k1].y * sn, col[k1].x * sn + col[k1].y * c);
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            Vt<T> row[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) row[n2] = y[k1 * R2 + n2];
            dftn<T, R2>(row, sg);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) u[k1 + R1 * k2] = row[k2];
        }
    }
}

// One Stockham stage of radix R over nb independent transforms of length n.
// Butterfly i (k = i mod p) reads positions i + q n/R, applies the twiddles
// exp(sg 2 pi i q k / (p R)), a length-R DFT, and writes positions
// (i - k) R + k + q p.  ROWL: element (pos, b) at b*n + pos, else pos*nb + b.
template <typename T, int R, bool ROWL>
__device__ __forceinline__ void stage(const Vt<T> *X, Vt<T> *Y, int n, int p, int nb,
                                      const Vt<T> *__restrict__ tw, T sg) {
    const int Tq = n / R;
    const int total = Tq * nb;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        int i, b;
        if (ROWL) {
            b = idx / Tq;
            i = idx - b * Tq;
        } else {
            i = idx / nb;
            b = idx - i * nb;
        }
        const int k = i % p;
        Vt<T> u[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int pos = i + q * Tq;
            u[q] = ROWL ? X[b * n + pos] : X[pos * nb + b];
        }
        if (p > 1) {
#pragma unroll
            for (int q = 1; q < R; ++q) {
                Vt<T> w = tw[(q - 1) * p + k];
                w.y *= -sg;  // table holds exp(-2 pi i q k / (p R))
                u[q] = cmul(u[q], w);
            }
        }
        dftn<T, R>(u, sg);
        const int j = (i - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int pos = j + q * p;
            if (ROWL)
                Y[b * n + pos] = u[q];
            else
                Y[pos * nb + b] = u[q];
        }
    }
}

// The stages of a transform of length f.L in LDS, ping-ponging between A and
// Bf; returns the buffer holding the result.
template <typename T, bool ROWL>
__device__ __forceinline__ Vt<T> *fft_stages(Vt<T> *A, Vt<T> *Bf, const FftDesc &f, int nb, const Vt<T> *tw, T sg,
                                              int tb = 0) {
    Vt<T> *X = A;
    Vt<T> *Y = Bf;
    int p = 1;
    for (int s = 0; s < f.nst; ++s) {
        const int r = f.radix[s];
        const Vt<T> *t = tw + (f.twoff[s] - tb);
        switch (r) {
            case 3: stage<T, 3, ROWL>(X, Y, f.L, p, nb, t, sg); break;
            case 5: stage<T, 5, ROWL>(X, Y, f.L, p, nb, t, sg); break;
            case 7: stage<T, 7, ROWL>(X, Y, f.L, p, nb, t, sg); break;
            case 9: stage<T, 9, ROWL>(X, Y, f.L, p, nb, t, sg); break;
            case 15: stage<T, 15, ROWL>(X, Y, f.L, p, nb, t, sg); break;
            default: stage<T, 25, ROWL>(X, Y, f.L, p, nb, t, sg); break;
        }
        __syncthreads();
        Vt<T> *tmp = X;
        X = Y;
        Y = tmp;
        p *= r;
    }
    return X;
}

// Full transform of nb sequences of length f.n in LDS (positions 0 .. n - 1 of
// buffers of f.L positions; ROWL: element (pos, b) at b L + pos, else
// pos nb + b); returns the buffer holding the result.  Must be called by
// every thread of the work-group.
template <typename T, bool ROWL>
__device__ __forceinline__ Vt<T> *fft_lds(Vt<T> *A, Vt<T> *Bf, const FftDesc &f, int nb, const Vt<T> *tw, T sg,
                                           int tb = 0) {
    if (!f.blue) return fft_stages<T, ROWL>(A, Bf, f, nb, tw, sg, tb);
    // Bluestein: u_j = x_j c_j zero-padded to L, H (.) DFT^- u, DFT^+, times c_k
    const int n = f.n, L = f.L;
    const Vt<T> *chirp = tw + (f.choff - tb);
    const Vt<T> *H = tw + (f.hoff - tb);
    auto at = [&](Vt<T> *buf, int pos, int b) -> Vt<T> & { return ROWL ? buf[b * L + pos] : buf[pos * nb + b]; };
    auto chirp_of = [&](int m) {  // c_m for the sign sg
        Vt<T> c = chirp[m];
        c.y *= sg;
        return c;
    };
    for (int idx = threadIdx.x; idx < L * nb; idx += blockDim.x) {
        const int b = idx / L, pos = idx - b * L;
        Vt<T> &v = at(A, pos, b);
        v = pos < n ? cmul(v, chirp_of(pos)) : mk<T>(T(0), T(0));
    }
    __syncthreads();
    Vt<T> *X = fft_stages<T, ROWL>(A, Bf, f, nb, tw, T(-1), tb);
    for (int idx = threadIdx.x; idx < L * nb; idx += blockDim.x) {
        const int b = idx / L, k = idx - b * L;
        // H for the sign sg: H_k (sg = +1) or conj(H_{-k}) (sg = -1)
        Vt<T> h = H[sg > T(0) ? k : (k == 0 ? 0 : L - k)];
        if (sg < T(0)) h.y = -h.y;
        Vt<T> &v = at(X, k, b);
        v = cmul(v, h);
    }
    __syncthreads();
    Vt<T> *Y = fft_stages<T, ROWL>(X, X == A ? Bf : A, f, nb, tw, T(1), tb);
    for (int idx = threadIdx.x; idx < n * nb; idx += blockDim.x) {
        const int b = idx / n, pos = idx - b * n;
        Vt<T> &v = at(Y, pos, b);
        v = cmul(v, chirp_of(pos));
    }
    __syncthreads();
    return Y;
}

// Deterministic work-group sum (fixed shuffle tree, then waves in order) over
// a work-group of at most NT threads; the result is valid in thread 0.
template <int NT>
__device__ double block_sum_t(double v) {
    __shared__ double red[NT / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    }
    __syncthreads();
    return s;
}
__device__ double block_sum(double v) { return block_sum_t<kThreads>(v); }

// K work-group sums at once, each in the order of block_sum (a shuffle tree
// per wave, then the waves in turn), written to out[0 .. K-1] by the first K
// threads: one barrier for all K instead of three per sum.
template <int K>
__device__ void block_sum_many(const double (&v)[K], double *out) {
    __shared__ double red[K][kThreads / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) red[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

__device__ __forceinline__ int wrapi(int i, int L) { return i < (L + 1) / 2 ? i : i - L; }
__device__ __forceinline__ int posmod(int k, int n) {
    int r = k % n;
    return r < 0 ? r + n : r;
}

// Orthonormal basis t_a(k) (a < nc) of the admissible directions at frequency k:
// primal (E_N): k/|k|; dual (J_N), d = 2: R k/|k| with R the rotation by +90
// degrees; d = 3: t1 = k x e_j / |k x e_j| with j the axis of smallest |k_j|
// (lowest index on ties) and t2 = s(k) k/|k| x t1 with s(k) the sign of the
// first non-zero k_j.  Every t_a is odd in k, so a field i sum_a t_a(k) c_a(k)
// is real exactly when each c_a is Hermitian.  Returns 0 at k = 0.
template <typename T>
__device__ __forceinline__ int basis(int d, int kind, int k1, int k2, int k3, T t[2][3]) {
    // straight-line code (selects, no branches): written per branch, the
    // compiler keeps the partially written rows of t on the stack
    // |k|^2 and |k x e_j|^2 are exact integers; rsqrt (reciprocal square
    // root, within a few ulp) replaces a square root and a division, and the
    // second one is only formed for the 3D dual (kind is uniform per launch)
    const T a = T(k1), b = T(k2), c = T(d == 3 ? k3 : 0);
    const T nn = a * a + b * b + c * c;
    const T inv = nn == T(0) ? T(0) : rsqrt(nn);
    const T h1 = a * inv, h2 = b * inv, h3 = c * inv;
    const int ab1 = k1 < 0 ? -k1 : k1, ab2 = k2 < 0 ? -k2 : k2, ab3 = k3 < 0 ? -k3 : k3;
    const bool x1 = ab1 <= ab2 && ab1 <= ab3;  // k x e_1
    const bool x2 = !x1 && ab2 <= ab3;         // k x e_2, else k x e_3
    T u1 = x1 ? T(0) : x2 ? -c : b;
    T u2 = x1 ? c : x2 ? T(0) : -a;
    T u3 = x1 ? -b : x2 ? a : T(0);
    const bool primal = kind == KIND_E, two = d == 2;
    T un = T(0);
    if (!primal && !two) {
        const T uu = u1 * u1 + u2 * u2 + u3 * u3;
        un = uu == T(0) ? T(0) : rsqrt(uu);
    }
    u1 *= un;
    u2 *= un;
    u3 *= un;
    const T s = (k1 != 0) ? (k1 > 0 ? T(1) : T(-1)) : (k2 != 0) ? (k2 > 0 ? T(1) : T(-1)) : (k3 > 0 ? T(1) : T(-1));
    t[0][0] = primal ? h1 : two ? -h2 : u1;
    t[0][1] = primal ? h2 : two ? h1 : u2;
    t[0][2] = primal ? h3 : two ? T(0) : u3;
    t[1][0] = s * (h2 * u3 - h3 * u2);
    t[1][1] = s * (h3 * u1 - h1 * u3);
    t[1][2] = s * (h1 * u2 - h2 * u1);
    return nn == T(0) ? 0 : (primal || two) ? 1 : 2;
}

// exp(-i pi sum_a s_a k_a / N_a) of the shift s (S(s) of Lemma reduce_grid);
// 1 when no shift is set.
__device__ __forceinline__ void shift_phase(const PencilArgs &a, int k1, int k2, int k3, double *c, double *s) {
    const double x = (a.shift[0] ? (double)k1 / a.Nfull[0] : 0.0) + (a.shift[1] ? (double)k2 / a.Nfull[1] : 0.0) +
                     (a.shift[2] ? (double)k3 / a.Nfull[2] : 0.0);
    sincospi(-x, s, c);
}
__device__ __forceinline__ bool has_shift(const PencilArgs &a) { return (a.shift[0] | a.shift[1] | a.shift[2]) != 0; }

__device__ __forceinline__ double sinc_pi(double x) {
    return x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x);
}

// ---------------------------------------------------------------------------
// Pencil pass: batched DFT along a strided axis.
// ---------------------------------------------------------------------------
// t[al] for a runtime component al < 3 without indexing a private array
template <typename T>
__device__ __forceinline__ T pick3(const T *t, int al) {
    return al == 0 ? t[0] : (al == 1 ? t[1] : t[2]);
}

// two waves per SIMD: the radix-25 stage alone would take the register
// file of one.  The components of a pencil are transformed a.cb at a time in
// one batch of cb * B sequences (layout: position * (cn B) + j B + b for
// component al0 + j of the chunk), so that a small grid runs one chain of
// stages and barriers per work-group instead of one per component.
template <typename T>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void pencil_kernel(PencilArgs a) {
    using V = Vt<T>;
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    const int n = a.f.n;
    const int B = a.B;
    const int cb = a.cb;
    V *bufA = reinterpret_cast<V *>(smem_raw);
    V *bufB = bufA + (size_t)a.f.L * cb * B;
    V *acc = bufB + (size_t)a.f.L * cb * B;
    const int b0 = blockIdx.x * B;
    const int o = blockIdx.y;
    const int nbw = min(B, a.nb - b0);
    const V *tw = reinterpret_cast<const V *>(a.tw);
    // the transform's table entries (stage twiddles; Bluestein chirp and
    // filter) staged in LDS after the buffers when they fit (a.twl entries from
    // entry twoff[0]); visible to the stages after the loads' barrier
    int tb = 0;
    if (a.twl > 0) {
        int lacc = 0;
        if (a.pro == PRO_EXPAND) lacc = a.nc * a.L_in;
        if (a.epi == EPI_PROJECT) lacc = a.nc * a.L_out;
        V *twl = acc + (size_t)lacc * B;
        tb = a.f.twoff[0];
        for (int i = threadIdx.x; i < a.twl; i += blockDim.x) twl[i] = tw[tb + i];
        tw = twl;
    }
    const T sg = T(a.sgn);
    const T scale = T(a.scale);
    const V *in = reinterpret_cast<const V *>(a.in);
    V *out = reinterpret_cast<V *>(a.out);
    const V zero = mk<T>(T(0), T(0));

    auto freq = [&](int l, int L, int b, int *k1, int *k2, int *k3) {
        *k1 = wrapi(l, L);
        if (a.d == 3) {
            *k2 = wrapi(b / a.Nh, a.Nmid);
            *k3 = b % a.Nh;
        } else {
            *k2 = b % a.Nh;
            *k3 = 0;
        }
    };

    if (a.pro == PRO_EXPAND) {
        // c_a -> e_alpha = i sum_a t_a(k)_alpha c_a on Z_N, zero-padded to n.
        const V *sr = reinterpret_cast<const V *>(a.st_r);
        V *sp = reinterpret_cast<V *>(a.st_p);
        const V *sx = reinterpret_cast<const V *>(a.st_x);
        const T beta = (a.update_p && a.status) ? T(a.status->beta) : T(0);
        for (int s = 0; s < a.nsol; ++s) {
            for (int idx = threadIdx.x; idx < a.nc * a.L_in * B; idx += blockDim.x) {
                const int bb = idx % B;
                const int l = (idx / B) % a.L_in;
                const int c = idx / (B * a.L_in);
                V v = zero;
                if (bb < nbw) {
                    const long off = s * a.st_ss + c * a.st_cs + (long)l * a.in_ls + b0 + bb;
                    if (a.update_p) {
                        const V r = sr[off];
                        const V pv = sp[off];
                        v = mk<T>(r.x + beta * pv.x, r.y + beta * pv.y);
                        sp[off] = v;
                    } else {
                        v = sx[off];
                    }
                }
                acc[(c * a.L_in + l) * B + bb] = v;
            }
            __syncthreads();
            for (int al0 = 0; al0 < a.ncomp; al0 += cb) {
                const int cn = min(cb, a.ncomp - al0);
                const int nbt = cn * B;
                for (int idx = threadIdx.x; idx < n * nbt; idx += blockDim.x) bufA[idx] = zero;
                __syncthreads();
                for (int idx = threadIdx.x; idx < a.L_in * B; idx += blockDim.x) {
                    const int bb = idx % B;
                    const int l = idx / B;
                    if (bb >= nbw) continue;
                    int k1, k2, k3;
                    freq(l, a.L_in, b0 + bb, &k1, &k2, &k3);
                    T t[2][3];
                    const int nt = basis<T>(a.d, a.kind, k1, k2, k3, t);
                    double pc = 1.0, ps = 0.0;
                    if (has_shift(a)) shift_phase(a, k1, k2, k3, &pc, &ps);
                    V *dst = bufA + posmod(k1, n) * nbt + bb;
                    for (int j = 0; j < cn; ++j) {
                        const int al = al0 + j;
                        T ex = T(0), ey = T(0);
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            if (c >= nt) break;
                            const V cv = acc[(c * a.L_in + l) * B + bb];
                            const T tc = pick3<T>(t[c], al);
                            ex -= tc * cv.y;  // i * t * c
                            ey += tc * cv.x;
                        }
                        if (has_shift(a)) {
                            const T nx = ex * T(pc) - ey * T(ps);
                            ey = ex * T(ps) + ey * T(pc);
                            ex = nx;
                        }
                        dst[j * B] = mk<T>(ex, ey);
                    }
                }
                __syncthreads();
                V *res = fft_lds<T, false>(bufA, bufB, a.f, nbt, tw, sg, tb);
                for (int idx = threadIdx.x; idx < a.L_out * nbt; idx += blockDim.x) {
                    const int bt = idx % nbt;
                    const int l = idx / nbt;
                    const int j = cn > 1 ? bt / B : 0;  // no division for one component
                    const int bb = bt - j * B;
                    if (bb >= nbw) continue;
                    const int pos = posmod(wrapi(l, a.L_out), n);
                    V v = res[pos * nbt + bt];
                    v.x *= scale;
                    v.y *= scale;
                    const long cbase = (long)(s * a.ncomp + al0 + j) * a.out_cs + (long)o * a.out_os + b0;
                    out[cbase + (long)l * a.out_ls + bb] = v;
                }
                __syncthreads();
            }
        }
        return;
    }

    // PRO_PLAIN
    if (a.epi == EPI_PROJECT) {
        for (int idx = threadIdx.x; idx < a.nc * a.L_out * B; idx += blockDim.x) acc[idx] = zero;
    }
    double part = 0.0;
    for (int al0 = 0; al0 < a.ncomp; al0 += cb) {
        const int cn = min(cb, a.ncomp - al0);
        const int nbt = cn * B;
        if (a.L_in < n) {
            for (int idx = threadIdx.x; idx < n * nbt; idx += blockDim.x) bufA[idx] = zero;
            __syncthreads();
        }
        for (int idx = threadIdx.x; idx < a.L_in * nbt; idx += blockDim.x) {
            const int bt = idx % nbt;
            const int l = idx / nbt;
            const int j = cn > 1 ? bt / B : 0;
            const int bb = bt - j * B;
            V v = zero;
            if (bb < nbw) v = in[(long)(al0 + j) * a.in_cs + (long)o * a.in_os + b0 + (long)l * a.in_ls + bb];
            bufA[posmod(wrapi(l, a.L_in), n) * nbt + bt] = v;
        }
        __syncthreads();
        V *res = fft_lds<T, false>(bufA, bufB, a.f, nbt, tw, sg, tb);
        if (a.epi == EPI_PROJECT) {
            // q_a += -i t_a(k)_alpha yhat_alpha(k) on Z_N, alpha in ascending order
            for (int idx = threadIdx.x; idx < a.L_out * B; idx += blockDim.x) {
                const int bb = idx % B;
                const int l = idx / B;
                if (bb >= nbw) continue;
                int k1, k2, k3;
                freq(l, a.L_out, b0 + bb, &k1, &k2, &k3);
                T t[2][3];
                const int nt = basis<T>(a.d, a.kind, k1, k2, k3, t);
                const V *src = res + posmod(k1, n) * nbt + bb;
                for (int j = 0; j < cn; ++j) {
                    const V y = src[j * B];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        if (c >= nt) break;
                        V &q = acc[(c * a.L_out + l) * B + bb];
                        const T tt = pick3<T>(t[c], al0 + j) * scale;
                        q.x += tt * y.y;
                        q.y -= tt * y.x;
                    }
                }
            }
        } else {
            for (int idx = threadIdx.x; idx < a.L_out * nbt; idx += blockDim.x) {
                const int bt = idx % nbt;
                const int l = idx / nbt;
                const int j = cn > 1 ? bt / B : 0;
                const int bb = bt - j * B;
                if (bb >= nbw) continue;
                const int kk = wrapi(l, a.L_out);
                V v = res[posmod(kk, n) * nbt + bt];
                T sc = scale;
                if (a.epi == EPI_WINDOW) {
                    int k1, k2, k3;
                    freq(l, a.L_out, b0 + bb, &k1, &k2, &k3);
                    double w = a.winscale * sinc_pi((double)k1 / a.Pw[0]) * sinc_pi((double)k2 / a.Pw[1]);
                    if (a.d == 3) w *= sinc_pi((double)k3 / a.Pw[2]);
                    sc = T(w * a.scale);
                }
                v.x *= sc;
                v.y *= sc;
                const long obase = (long)(al0 + j) * a.out_cs + (long)o * a.out_os + b0;
                out[obase + (long)l * a.out_ls + bb] = v;
            }
        }
        __syncthreads();
    }
    if (a.epi == EPI_PROJECT) {
        V *q = out;
        const V *dv = reinterpret_cast<const V *>(a.st_dot);
        for (int idx = threadIdx.x; idx < a.nc * a.L_out * B; idx += blockDim.x) {
            const int bb = idx % B;
            const int l = (idx / B) % a.L_out;
            const int c = idx / (B * a.L_out);
            if (bb >= nbw) continue;
            V v = acc[idx];
            const long off = (long)c * a.out_cs + (long)l * a.out_ls + b0 + bb;
            if (has_shift(a)) {  // S*(s): the conjugate phase
                int k1, k2, k3;
                freq(l, a.L_out, b0 + bb, &k1, &k2, &k3);
                double pc, ps;
                shift_phase(a, k1, k2, k3, &pc, &ps);
                const T nx = v.x * T(pc) + v.y * T(ps);
                v.y = v.y * T(pc) - v.x * T(ps);
                v.x = nx;
            }
            if (a.accumulate) {
                const V old = q[off];
                v.x += old.x;
                v.y += old.y;
            }
            q[off] = v;
            const int klast = (b0 + bb) % a.Nh;
            const double w = klast == 0 ? 1.0 : 2.0;
            if (dv != nullptr) {
                const V pv = dv[off];
                part += w * ((double)pv.x * (double)v.x + (double)pv.y * (double)v.y);
            } else {
                part += w * ((double)v.x * (double)v.x + (double)v.y * (double)v.y);
            }
        }
        const double s = block_sum(part);
        if (threadIdx.x == 0) a.partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// Voxel value as seen by the material series: the conductivity itself (0), the
// indicator of the high phase of a two-phase image (1), the inverse
// conductivity (2), or zero (3, a one-phase image).
template <typename T>
__device__ __forceinline__ T map_voxel(T v, int mode, double vmax) {
    if (mode == 1) return v == T(vmax) ? T(1) : T(0);
    if (mode == 2) return T(1) / v;
    if (mode == 3) return T(0);
    return v;
}

// GaNi material (Def. GaNi: the rectangle rule samples A at the grid points).
__global__ __launch_bounds__(kThreads) void sample_incl_kernel(double *g, int d, int m0, int m1, int m2,
                                                               const InclDev *inc, int n, double w0) {
    const long total = (long)m0 * m1 * m2;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kThreads) {
        const int j2 = (int)(idx % m2);
        const int j1 = (int)((idx / m2) % m1);
        const int j0 = (int)(idx / ((long)m2 * m1));
        double x[3];
        x[0] = (double)wrapi(j0, m0) / m0;
        x[1] = (double)wrapi(j1, m1) / m1;
        x[2] = (double)wrapi(j2, m2) / m2;  // 2D: m2 = 1, x[2] unused
        double v = w0;
        for (int i = 0; i < n; ++i) {
            double r2 = 0.0;
            bool inside = true;
            for (int a = 0; a < d; ++a) {
                double dx = x[a] - inc[i].c[a];
                dx -= rint(dx);
                if (inc[i].shape == 0)
                    inside = inside && fabs(dx) < 0.5 * inc[i].h[a];
                else
                    r2 += dx * dx;
            }
            if (inc[i].shape != 0) inside = r2 < inc[i].h[0] * inc[i].h[0];
            if (inside) v += inc[i].w;
        }
        g[idx] = v;
    }
}

__global__ __launch_bounds__(kThreads) void sample_voxel_kernel(double *g, const double *img, int p0, int p1, int p2,
                                                                int m0, int m1, int m2, int map, double vmax) {
    const long total = (long)m0 * m1 * m2;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kThreads) {
        const int j2 = (int)(idx % m2);
        const int j1 = (int)((idx / m2) % m1);
        const int j0 = (int)(idx / ((long)m2 * m1));
        const int q0 = posmod((int)rint((double)wrapi(j0, m0) * p0 / m0), p0);
        const int q1 = posmod((int)rint((double)wrapi(j1, m1) * p1 / m1), p1);
        const int q2 = posmod((int)rint((double)wrapi(j2, m2) * p2 / m2), p2);
        g[idx] = map_voxel<double>(img[((long)q0 * p1 + q1) * p2 + q2], map, vmax);
    }
}

// Upper and lower voxel images (Remark adjusting_A).
__global__ __launch_bounds__(kThreads) void envelope_kernel(double *up, double *lo, int d, int p0, int p1, int p2,
                                                            const InclDev *inc, int n, const double *ext) {
    const long total = (long)p0 * p1 * p2;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kThreads) {
        const int j2 = (int)(idx % p2);
        const int j1 = (int)((idx / p2) % p1);
        const int j0 = (int)(idx / ((long)p2 * p1));
        const int pp[3] = {p0, p1, p2};
        const double x[3] = {(double)wrapi(j0, p0) / p0, (double)wrapi(j1, p1) / p1, (double)wrapi(j2, p2) / p2};
        double hi = -HUGE_VAL, lw = HUGE_VAL;
        bool matrix = true;
        for (int i = 0; i < n; ++i) {
            bool meets = true, contains = true;
            double near2 = 0.0, far2 = 0.0;
            for (int a = 0; a < d; ++a) {
                double dc = x[a] - inc[i].c[a];
                dc = fabs(dc - rint(dc));
                const double half = 0.5 / pp[a];
                if (inc[i].shape == 0) {
                    meets = meets && dc < 0.5 * inc[i].h[a] + half;
                    contains = contains && dc + half <= 0.5 * inc[i].h[a];
                } else {
                    // unfused, so that a voxel exactly on the circle is classified
                    // as in plain rounded arithmetic
                    const double nr = fmax(dc - half, 0.0), fr = dc + half;
                    near2 = __dadd_rn(near2, __dmul_rn(nr, nr));
                    far2 = __dadd_rn(far2, __dmul_rn(fr, fr));
                }
            }
            if (inc[i].shape != 0) {
                const double r2 = __dmul_rn(inc[i].h[0], inc[i].h[0]);
                meets = near2 < r2;
                contains = far2 <= r2;
            }
            if (meets) {
                hi = fmax(hi, ext[2 + 2 * i]);
                lw = fmin(lw, ext[3 + 2 * i]);
            }
            if (contains) matrix = false;
        }
        if (matrix) {
            hi = fmax(hi, ext[0]);
            lw = fmin(lw, ext[1]);
        }
        up[idx] = hi;
        lo[idx] = lw;
    }
}

// Reduced Ga material: fold the series on Z_{2N-1} onto Z_N with the phase of
// shift s (one output frequency per thread; at most two sources per axis).
// Index 2 is always the last axis; index 1 is used in 3D only.
__global__ __launch_bounds__(kThreads) void fold_series_kernel(double2 *out, const double2 *coef, int d, int n0,
                                                               int n1, int n2, int l0, int l1, int lh, int s0, int s1,
                                                               int s2) {
    const int nh = (n2 + 1) / 2;  // stored output entries along the last axis
    const long total = (d == 3 ? (long)n0 * n1 : (long)n0) * nh;
    const int nn[3] = {n0, n1, n2};
    const int sh[3] = {s0, d == 3 ? s1 : 0, s2};
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kThreads) {
        const int m2 = (int)(idx % nh);
        const long r = idx / nh;
        const int m1 = d == 3 ? (int)(r % n1) : 0;
        const int m0 = d == 3 ? (int)(r / n1) : (int)r;
        const int jj[3] = {wrapi(m0, n0), d == 3 ? wrapi(m1, n1) : 0, m2};
        // sources k_a = j_a and j_a -/+ N_a (for j_a != 0): |k_a| <= N_a - 1
        int ka[3][2], na[3];
        for (int a = 0; a < 3; ++a) {
            ka[a][0] = jj[a];
            ka[a][1] = jj[a] > 0 ? jj[a] - nn[a] : jj[a] + nn[a];
            na[a] = (jj[a] != 0 && (a != 1 || d == 3)) ? 2 : 1;
        }
        double re = 0.0, im = 0.0;
        for (int i0 = 0; i0 < na[0]; ++i0)
            for (int i1 = 0; i1 < na[1]; ++i1)
                for (int i2 = 0; i2 < na[2]; ++i2) {
                    const int k0 = ka[0][i0], k1 = ka[1][i1], k2 = ka[2][i2];
                    // stored entries have k_last >= 0; the others by conjugate symmetry
                    const bool cj = k2 < 0;
                    const int q0 = cj ? -k0 : k0, q1 = cj ? -k1 : k1, q2 = cj ? -k2 : k2;
                    double2 v = d == 3 ? coef[((long)posmod(q0, l0) * l1 + posmod(q1, l1)) * lh + q2]
                                       : coef[(long)posmod(q0, l0) * lh + q2];
                    if (cj) v.y = -v.y;
                    const double x = (sh[0] ? (double)k0 / nn[0] : 0.0) + (sh[1] ? (double)k1 / nn[1] : 0.0) +
                                     (sh[2] ? (double)k2 / nn[2] : 0.0);
                    double ps, pc;
                    sincospi(-x, &ps, &pc);
                    re += v.x * pc - v.y * ps;
                    im += v.x * ps + v.y * pc;
                }
        out[idx] = make_double2(re, im);
    }
}

// Symmetric material matrix at linear grid point pt from d (d + 1) / 2 fields
// (entries 11, 12, [13,] 22, [23,] 33; field f at g + f * stride).
template <typename T>
__device__ __forceinline__ void sym_load(const T *g, long stride, long pt, int d, T *m) {
    int f = 0;
    for (int i = 0; i < d; ++i)
        for (int j = i; j < d; ++j) {
            const T v = g[(long)f * stride + pt];
            m[i * d + j] = v;
            m[j * d + i] = v;
            ++f;
        }
}

// ---------------------------------------------------------------------------
// Row pass: real transforms along the last axis, two rows per complex DFT.
// ---------------------------------------------------------------------------
// Transform buffers (components) of the generic row kernel.
__host__ __device__ inline int row_zbufs(const RowArgs &a) {
    if (a.mode == ROW_RHS) return a.d;
    if (a.mode == ROW_R2C || a.mode == ROW_C2R) return 1;
    if (a.mode == ROW_GRAM && a.gpack) return (a.ncomp + 1) / 2;
    return a.ncomp;
}

template <typename T, int DIM>
__global__ __launch_bounds__(kThreads) void row_kernel(RowArgs a) {
    using V = Vt<T>;
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    const int n = a.f.n;
    const int ln = a.f.L;  // buffer length per transform (n unless Bluestein)
    const int RP = a.RP;
    const int nh = a.Nh_row;
    // one buffer per component (Z[c] = Z + c RP ln) and the transforms'
    // scratch S: RP ln (a batch per component) or the size of Z (zbatch: the
    // rows of all components form one batch, sequence c RP + j at (c RP + j) ln)
    const bool zb = a.zbatch != 0;
    const int nzb = row_zbufs(a);
    V *const S = reinterpret_cast<V *>(smem_raw) + (zb ? (size_t)nzb * RP * ln : 0);
    V *const Z = reinterpret_cast<V *>(smem_raw) + (zb ? 0 : (size_t)RP * ln);
    const V *tw = reinterpret_cast<const V *>(a.tw);
    V *data = reinterpret_cast<V *>(a.data);
    const T *g = reinterpret_cast<const T *>(a.g);
    const int pair0 = blockIdx.x * RP;
    const int npairs_total = (a.nrows + 1) / 2;
    const int nvp = min(RP, npairs_total - pair0);
    const V zero = mk<T>(T(0), T(0));
    constexpr int d = DIM;  // the material and field loops unroll (no private arrays)
    const int nzc = (a.mode == ROW_RHS || a.mode == ROW_R2C) ? (a.mode == ROW_RHS ? d : 1) : a.ncomp;

    auto zbuf = [&](int c) { return Z + (size_t)c * RP * ln; };
    auto fft_into = [&](int c, T sg) {
        V *res = fft_lds<T, true>(zbuf(c), S, a.f, RP, tw, sg);
        if (res != zbuf(c)) {
            for (int idx = threadIdx.x; idx < RP * ln; idx += blockDim.x) zbuf(c)[idx] = res[idx];
            __syncthreads();
        }
    };

    if (a.mode == ROW_GRAM && a.gpack) {
        // (A_M (E_s + e_s), E_t + e_t) with components 2 c2 and 2 c2 + 1 of one
        // row packed per transform (z = u_{2 c2} + i u_{2 c2 + 1}); row r0 + j
        const int r0 = blockIdx.x * RP;
        const int nvr = min(RP, a.nrows - r0);
        const int npk = (a.ncomp + 1) / 2;
        for (int c2 = 0; c2 < npk; ++c2) {
            V *zc = zbuf(c2);
            for (int idx = threadIdx.x; idx < RP * ln; idx += blockDim.x) zc[idx] = zero;
            __syncthreads();
            const bool two = 2 * c2 + 1 < a.ncomp;
            for (int idx = threadIdx.x; idx < RP * nh; idx += blockDim.x) {
                const int j = idx / nh;
                const int kx = idx - j * nh;
                if (j >= nvr) continue;
                const long row = (long)(r0 + j) * nh + kx;
                const V u1 = data[(long)(2 * c2) * a.cs + row];
                const V u2 = two ? data[(long)(2 * c2 + 1) * a.cs + row] : mk<T>(T(0), T(0));
                if (kx == 0) {
                    zc[j * ln] = mk<T>(u1.x, u2.x);
                } else {
                    zc[j * ln + kx] = mk<T>(u1.x - u2.y, u1.y + u2.x);
                    zc[j * ln + n - kx] = mk<T>(u1.x + u2.y, u2.x - u1.y);
                }
            }
            __syncthreads();
            fft_into(c2, T(1));
        }
        T A0[9], D[9];
        for (int i = 0; i < d * d; ++i) {
            A0[i] = T(a.A0[i]);
            D[i] = T(a.D[i]);
        }
        double gs[9];
        for (int i = 0; i < 9; ++i) gs[i] = 0.0;
        for (int idx = threadIdx.x; idx < RP * n; idx += blockDim.x) {
            const int j = idx / n;
            const int x = idx - j * n;
            if (j >= nvr) continue;
            const long r = r0 + j;
            T am[9];
            if (a.nfield > 1) {
                sym_load<T>(g, a.gstride, r * n + x, d, am);
            } else {
                const T gg = g[r * n + x];
                for (int i = 0; i < d * d; ++i) am[i] = A0[i] + gg * D[i];
            }
            T f[3][3];
            for (int s2 = 0; s2 < d; ++s2)
                for (int b = 0; b < d; ++b) {
                    const int c = s2 * d + b;
                    const V zv = zbuf(c / 2)[j * ln + x];
                    f[s2][b] = ((c & 1) ? zv.y : zv.x) + (s2 == b ? T(1) : T(0));
                }
            for (int t = 0; t < d; ++t) {
                T af[3];
                for (int al = 0; al < d; ++al) {
                    T y = T(0);
                    for (int b = 0; b < d; ++b) y += am[al * d + b] * f[t][b];
                    af[al] = y;
                }
                for (int s2 = 0; s2 < d; ++s2) {
                    T dot = T(0);
                    for (int al = 0; al < d; ++al) dot += f[s2][al] * af[al];
                    gs[s2 * d + t] += dot;
                }
            }
        }
        for (int i = 0; i < d * d; ++i) {
            const double sum = block_sum(gs[i]);
            if (threadIdx.x == 0) a.partial[(long)blockIdx.x * d * d + i] = sum;
        }
        return;
    }

    // ---- spatial values ----
    if (zb && (a.mode == ROW_OPER || a.mode == ROW_GRAM || a.mode == ROW_C2R)) {
        const int nall = a.ncomp * RP;
        for (int idx = threadIdx.x; idx < nall * ln; idx += blockDim.x) Z[idx] = zero;
        __syncthreads();
        for (int idx = threadIdx.x; idx < nall * nh; idx += blockDim.x) {
            const int cj = idx / nh;  // c RP + j
            const int kx = idx - cj * nh;
            const int c = cj / RP;
            const int j = cj - c * RP;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            const V u1 = data[(long)c * a.cs + (long)r1 * nh + kx];
            const V u2 = (r2 < a.nrows) ? data[(long)c * a.cs + (long)r2 * nh + kx] : mk<T>(T(0), T(0));
            V *zr = Z + (size_t)cj * ln;
            if (kx == 0) {
                zr[0] = mk<T>(u1.x, u2.x);
            } else {
                zr[kx] = mk<T>(u1.x - u2.y, u1.y + u2.x);
                zr[n - kx] = mk<T>(u1.x + u2.y, u2.x - u1.y);
            }
        }
        __syncthreads();
        const V *res = fft_lds<T, true>(Z, S, a.f, nall, tw, T(1));
        if (res != Z) {
            for (int idx = threadIdx.x; idx < nall * ln; idx += blockDim.x) Z[idx] = res[idx];
            __syncthreads();
        }
    } else if (a.mode == ROW_OPER || a.mode == ROW_GRAM || a.mode == ROW_C2R) {
        for (int c = 0; c < a.ncomp; ++c) {
            V *zc = zbuf(c);
            for (int idx = threadIdx.x; idx < RP * ln; idx += blockDim.x) zc[idx] = zero;
            __syncthreads();
            for (int idx = threadIdx.x; idx < RP * nh; idx += blockDim.x) {
                const int j = idx / nh;
                const int kx = idx - j * nh;
                if (j >= nvp) continue;
                const int r1 = 2 * (pair0 + j);
                const int r2 = r1 + 1;
                const V u1 = data[(long)c * a.cs + (long)r1 * nh + kx];
                const V u2 = (r2 < a.nrows) ? data[(long)c * a.cs + (long)r2 * nh + kx] : mk<T>(T(0), T(0));
                if (kx == 0) {
                    zc[j * ln] = mk<T>(u1.x, u2.x);
                } else {
                    zc[j * ln + kx] = mk<T>(u1.x - u2.y, u1.y + u2.x);
                    zc[j * ln + n - kx] = mk<T>(u1.x + u2.y, u2.x - u1.y);
                }
            }
            __syncthreads();
            fft_into(c, T(1));
        }
    } else if (a.mode == ROW_R2C) {
        const T *rin = reinterpret_cast<const T *>(a.real_in);
        V *zc = zbuf(0);
        for (int idx = threadIdx.x; idx < RP * n; idx += blockDim.x) {
            const int j = idx / n;
            const int x = idx - j * n;
            V v = zero;
            if (j < nvp) {
                const int r1 = 2 * (pair0 + j);
                const int r2 = r1 + 1;
                v.x = map_voxel<T>(rin[(long)r1 * a.real_stride + x], a.imgmap, a.vmax);
                v.y = (r2 < a.nrows) ? map_voxel<T>(rin[(long)r2 * a.real_stride + x], a.imgmap, a.vmax) : T(0);
            }
            zc[j * ln + x] = v;
        }
        __syncthreads();
    }

    // ---- pointwise work ----
    if (a.mode == ROW_OPER || a.mode == ROW_RHS) {
        T A0[9], D[9], E[3];
        for (int i = 0; i < d * d; ++i) {
            A0[i] = T(a.A0[i]);
            D[i] = T(a.D[i]);
        }
        for (int i = 0; i < 3; ++i) E[i] = T(a.E[i]);
        double load = 0.0, work = 0.0;
        for (int idx = threadIdx.x; idx < RP * n; idx += blockDim.x) {
            const int j = idx / n;
            const int x = idx - j * n;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            const bool v2 = r2 < a.nrows;
            T m1[9], m2[9];
            if (a.nfield > 1) {
                sym_load<T>(g, a.gstride, (long)r1 * n + x, d, m1);
                if (v2)
                    sym_load<T>(g, a.gstride, (long)r2 * n + x, d, m2);
                else
                    for (int i = 0; i < d * d; ++i) m2[i] = T(0);
            } else {
                const T g1 = g[(long)r1 * n + x];
                const T g2 = v2 ? g[(long)r2 * n + x] : T(0);
                for (int i = 0; i < d * d; ++i) {
                    m1[i] = A0[i] + g1 * D[i];
                    m2[i] = A0[i] + g2 * D[i];
                }
            }
            T e1[3], e2[3];
            for (int b = 0; b < d; ++b) {
                if (a.mode == ROW_OPER) {
                    const V zv = zbuf(b)[j * ln + x];
                    e1[b] = zv.x;
                    e2[b] = zv.y;
                } else {
                    e1[b] = E[b];
                    e2[b] = v2 ? E[b] : T(0);
                }
            }
            for (int al = 0; al < d; ++al) {
                T y1 = T(0), y2 = T(0);
                for (int b = 0; b < d; ++b) {
                    y1 += m1[al * d + b] * e1[b];
                    y2 += m2[al * d + b] * e2[b];
                }
                zbuf(al)[j * ln + x] = mk<T>(y1, y2);
                load += (double)y1 * y1 + (double)y2 * y2;
                if (a.mode == ROW_RHS) work += ((double)y1 + (double)y2) * a.E[al];
            }
        }
        __syncthreads();
        if (a.mode == ROW_RHS) {
            const double s = block_sum(load);
            const double s2 = block_sum(work);
            if (threadIdx.x == 0) {
                a.partial[blockIdx.x] = s;
                if (a.partial2 != nullptr) a.partial2[blockIdx.x] = s2;
            }
        }
    } else if (a.mode == ROW_GRAM) {
        // (A_M (E_s + e_s), E_t + e_t) summed over the rows' grid points
        T A0[9], D[9];
        for (int i = 0; i < d * d; ++i) {
            A0[i] = T(a.A0[i]);
            D[i] = T(a.D[i]);
        }
        double gs[9];
        for (int i = 0; i < 9; ++i) gs[i] = 0.0;
        for (int idx = threadIdx.x; idx < RP * n; idx += blockDim.x) {
            const int j = idx / n;
            const int x = idx - j * n;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            for (int half = 0; half < 2; ++half) {
                const int r = half ? r2 : r1;
                if (r >= a.nrows) continue;
                T am[9];
                if (a.nfield > 1) {
                    sym_load<T>(g, a.gstride, (long)r * n + x, d, am);
                } else {
                    const T gg = g[(long)r * n + x];
                    for (int i = 0; i < d * d; ++i) am[i] = A0[i] + gg * D[i];
                }
                T f[3][3];
                for (int s = 0; s < d; ++s)
                    for (int b = 0; b < d; ++b) {
                        const V zv = zbuf(s * d + b)[j * ln + x];
                        f[s][b] = (half ? zv.y : zv.x) + (s == b ? T(1) : T(0));
                    }
                for (int t = 0; t < d; ++t) {
                    T af[3];
                    for (int al = 0; al < d; ++al) {
                        T y = T(0);
                        for (int b = 0; b < d; ++b) y += am[al * d + b] * f[t][b];
                        af[al] = y;
                    }
                    for (int s = 0; s < d; ++s) {
                        T dot = T(0);
                        for (int al = 0; al < d; ++al) dot += f[s][al] * af[al];
                        gs[s * d + t] += dot;
                    }
                }
            }
        }
        for (int i = 0; i < d * d; ++i) {
            const double s = block_sum(gs[i]);
            if (threadIdx.x == 0) a.partial[(long)blockIdx.x * d * d + i] = s;
        }
        return;
    } else if (a.mode == ROW_C2R) {
        T *rout = reinterpret_cast<T *>(a.real_out);
        const T scale = T(a.scale);
        for (int idx = threadIdx.x; idx < RP * n; idx += blockDim.x) {
            const int j = idx / n;
            const int x = idx - j * n;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            const V zv = zbuf(0)[j * ln + x];
            rout[(long)r1 * a.real_stride + x] = zv.x * scale;
            if (r2 < a.nrows) rout[(long)r2 * a.real_stride + x] = zv.y * scale;
        }
        return;
    }

    // ---- forward transforms and Hermitian split ----
    const T half = T(a.scale) * T(0.5);
    if (zb) {
        const V *res = fft_lds<T, true>(Z, S, a.f, nzc * RP, tw, T(-1));
        for (int idx = threadIdx.x; idx < nzc * RP * nh; idx += blockDim.x) {
            const int cj = idx / nh;
            const int kx = idx - cj * nh;
            const int c = cj / RP;
            const int j = cj - c * RP;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            const V *zr = res + (size_t)cj * ln;
            const V w = zr[posmod(kx, n)];
            const V wm = zr[posmod(-kx, n)];
            data[(long)c * a.cs + (long)r1 * nh + kx] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
            if (r2 < a.nrows)
                data[(long)c * a.cs + (long)r2 * nh + kx] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
        }
        return;
    }
    for (int c = 0; c < nzc; ++c) {
        fft_into(c, T(-1));
        const V *zc = zbuf(c);
        for (int idx = threadIdx.x; idx < RP * nh; idx += blockDim.x) {
            const int j = idx / nh;
            const int kx = idx - j * nh;
            if (j >= nvp) continue;
            const int r1 = 2 * (pair0 + j);
            const int r2 = r1 + 1;
            const V w = zc[j * ln + posmod(kx, n)];
            const V wm = zc[j * ln + posmod(-kx, n)];
            data[(long)c * a.cs + (long)r1 * nh + kx] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
            if (r2 < a.nrows)
                data[(long)c * a.cs + (long)r2 * nh + kx] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// CG scalar and vector kernels (Remark CG; Saad Alg. 6.18).
// ---------------------------------------------------------------------------
// Sum of n partials in a fixed order: thread t adds entries t, t + blockDim,
// t + 2 blockDim, ... in turn, then block_sum; the loads of eight such steps
// are issued together (an entry past n adds an exact zero).
__device__ double sum_fixed(const double *part, int n) {
    constexpr int G = 8;
    double v = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += G * blockDim.x) {
        double t[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const int i = i0 + j * (int)blockDim.x;
            t[j] = i < n ? part[i] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < G; ++j) v += t[j];
    }
    return block_sum(v);
}

// hist[0] = (r_0, r_0); hist[1] = the energy (A_M E, E) of the initial iterate
// e_0 = 0 (the Voigt entry), from the right-hand side pass's sums of (A_M E).E.
__global__ __launch_bounds__(kThreads) void cg_init_kernel(CgStatus *st, const double *rr_part, int n_rr,
                                                           const double *load_part, int n_load,
                                                           const double *work_part, double inv_mtot, double tol,
                                                           double floor_rel, int maxit, double btol, double *hist) {
    const double rr = sum_fixed(rr_part, n_rr);
    const double load = sum_fixed(load_part, n_load);
    const double work = work_part != nullptr ? sum_fixed(work_part, n_load) : 0.0;
    if (threadIdx.x == 0) {
        st->rr = rr;
        st->rr0 = rr;
        st->pq = 0.0;
        st->alpha = 0.0;
        st->beta = 0.0;
        st->tol2 = tol * tol;
        st->load2 = load;
        st->floor2 = floor_rel * floor_rel * load;
        st->iter = 0;
        st->maxit = maxit;
        st->energy = work * inv_mtot;
        st->dprev = 0.0;
        st->btol = btol;
        st->eAE = st->energy;
        st->ebest = st->energy;  // e_0 = 0: the kept copy starts as zero
        st->rrmin = rr;
        st->rrmin_it = 0;
        st->best_it = 0;
        st->stagnated = 0;
        st->ck_copy = 0;
        st->ck_restore = 0;
        st->breakdown = !isfinite(rr) || !isfinite(load);
        st->converged = (rr == 0.0 || rr <= st->floor2) && !st->breakdown;
        st->done = st->converged || st->breakdown || maxit <= 0;
        if (hist != nullptr) {
            hist[0] = rr;
            hist[1] = st->energy;
        }
    }
}

// Warm start from an admissible initial iterate x0 (Remark CG: CG from an
// initial approximation in the minimisation space): r_0 = b - K x0 with r
// holding b and q = K x0 on entry; partial sums of (r_0, r_0), (b, x0) and
// (r_0, x0) in the weights of the half-spectrum storage.
template <typename T>
__global__ __launch_bounds__(kThreads) void warm_residual_kernel(UpdArgs a, double *part_rr, double *part_bx,
                                                                 double *part_rx) {
    Vt<T> *r = reinterpret_cast<Vt<T> *>(a.r);
    const Vt<T> *x = reinterpret_cast<const Vt<T> *>(a.x);
    const Vt<T> *q = reinterpret_cast<const Vt<T> *>(a.q);
    double prr = 0.0, pbx = 0.0, prx = 0.0;
    const long total = a.n_per_comp * a.nc;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)a.nblocks * kThreads) {
        const long c = idx / a.n_per_comp;
        const long i = idx - c * a.n_per_comp;
        const long off = c * a.cs + i;
        const Vt<T> bv = r[off], qv = q[off], xv = x[off];
        Vt<T> rv = bv;
        rv.x -= qv.x;
        rv.y -= qv.y;
        r[off] = rv;
        const double w = (i % a.Nh) == 0 ? 1.0 : 2.0;
        prr += w * ((double)rv.x * rv.x + (double)rv.y * rv.y);
        pbx += w * ((double)bv.x * xv.x + (double)bv.y * xv.y);
        prx += w * ((double)rv.x * xv.x + (double)rv.y * xv.y);
    }
    const double s1 = block_sum(prr);
    const double s2 = block_sum(pbx);
    const double s3 = block_sum(prx);
    if (threadIdx.x == 0) {
        part_rr[blockIdx.x] = s1;
        part_bx[blockIdx.x] = s2;
        part_rx[blockIdx.x] = s3;
    }
}

// Energy at x0: (A(E + x0), E + x0) = (A E, E) + 2 phi(x0), phi(x) =
// (K x, x) / 2 - (b, x), and (K x0, x0) = (b - r_0, x0).
__global__ __launch_bounds__(kThreads) void cg_init_warm_kernel(CgStatus *st, const double *part_rr,
                                                                const double *part_bx, const double *part_rx,
                                                                int nparts, const double *scal, double mtot,
                                                                double tol, double floor_rel, int maxit, double btol,
                                                                double *hist) {
    const double rr = sum_fixed(part_rr, nparts);
    const double bx = sum_fixed(part_bx, nparts);
    const double rx = sum_fixed(part_rx, nparts);
    if (threadIdx.x == 0) {
        const double bb = scal[0];
        const double load = scal[1];
        st->rr = rr;
        st->rr0 = bb;
        st->pq = 0.0;
        st->alpha = 0.0;
        st->beta = 0.0;
        st->tol2 = tol * tol;
        st->load2 = load;
        st->floor2 = floor_rel * floor_rel * load;
        st->iter = 0;
        st->maxit = maxit;
        st->energy = scal[2] / mtot - bx - rx;
        st->dprev = 0.0;
        st->btol = btol;
        st->eAE = scal[2] / mtot;
        st->ebest = st->energy;  // the kept copy starts as the initial iterate
        st->rrmin = rr;
        st->rrmin_it = 0;
        st->best_it = 0;
        st->stagnated = 0;
        st->ck_copy = 0;
        st->ck_restore = 0;
        st->breakdown = !isfinite(rr) || !isfinite(load) || !isfinite(bb);
        st->converged = (rr == 0.0 || rr <= st->tol2 * bb || rr <= st->floor2) && !st->breakdown;
        st->done = st->converged || st->breakdown || maxit <= 0;
        if (hist != nullptr) {
            hist[0] = rr;
            hist[1] = st->energy;
        }
    }
}

// Prolongation of the coefficients of a coarse solve (grid Nc) to a fine one
// (grid Nf): the trigonometric polynomial is kept (Fourier zero padding), so
// the entries of frequencies k in Z_Nc move and all others are zero.  Storage
// [c][k1][k2][k3 >= 0] (2D: [c][k1][k2 >= 0]) with wrapped indices.
template <typename TS, typename TD>
__global__ __launch_bounds__(kThreads) void prolong_kernel(const Vt<TS> *src, Vt<TD> *dst, int d, int nc, int f1,
                                                           int f2, int f3h, int c1, int c2, int c3h) {
    const long nsf = (long)f1 * f2 * f3h;  // 2D: f2 = 1
    const long nsc = (long)c1 * c2 * c3h;
    const long total = nsf * nc;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)gridDim.x * kThreads) {
        const long c = idx / nsf;
        long rem = idx - c * nsf;
        const int i3 = (int)(rem % f3h);
        rem /= f3h;
        const int i2 = (int)(rem % f2);
        const int i1 = (int)(rem / f2);
        const int k1 = wrapi(i1, f1);
        const int k2 = d == 3 ? wrapi(i2, f2) : 0;
        const bool in = (k1 >= -(c1 / 2) && k1 < (c1 + 1) / 2) && (d == 2 || (k2 >= -(c2 / 2) && k2 < (c2 + 1) / 2)) &&
                        i3 < c3h;
        Vt<TD> v;
        v.x = TD(0);
        v.y = TD(0);
        if (in) {
            const long j = ((long)posmod(k1, c1) * c2 + (d == 3 ? posmod(k2, c2) : 0)) * c3h + i3;
            const Vt<TS> u = src[c * nsc + j];
            v.x = TD(u.x);
            v.y = TD(u.y);
        }
        dst[idx] = v;
    }
}




__global__ void fill_zero_kernel(unsigned int *p, size_t nwords) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void f2d_kernel(double *dst, const float *src, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

__global__ void d2f_kernel(float *dst, const double *src, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// out[v] = sum_i part[i * nvals + v] in a fixed order (work-group v).
__global__ __launch_bounds__(kThreads) void sum_partials_kernel(double *out, const double *part, int nparts,
                                                                int nvals) {
    const int v = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[(long)i * nvals + v];
    s = block_sum(s);
    if (threadIdx.x == 0) out[v] = s;
}

// Fourier coefficients on the half grid of Z_{L} (L = 2N-1): entry
// (n_1, [n_2,] n_3 >= 0) = w0 [n = 0] + sum_i w_i exp(-2 pi i n.c_i) fhat_i(n),
// with fhat of the box prod_a h_a sinc(h_a n_a) or of the disc
// r J_1(2 pi r |n|)/|n| (pi r^2 at n = 0)  (eq. char_func_Four, eq. inclcomp_formula).
__global__ __launch_bounds__(kThreads) void incl_coeff_kernel(double2 *out, int d, int L1, int L2, int Lh,
                                                              const InclDev *incl, int n_incl, double w0) {
    const long total = (d == 3 ? (long)L1 * L2 * Lh : (long)L1 * Lh);
    for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total; idx += (long)gridDim.x * blockDim.x) {
        int n1, n2, n3;
        if (d == 3) {
            n3 = (int)(idx % Lh);
            n2 = wrapi((int)((idx / Lh) % L2), L2);
            n1 = wrapi((int)(idx / ((long)Lh * L2)), L1);
        } else {
            n3 = 0;
            n2 = (int)(idx % Lh);
            n1 = wrapi((int)(idx / Lh), L1);
        }
        double re = (n1 == 0 && n2 == 0 && n3 == 0) ? w0 : 0.0, im = 0.0;
        for (int i = 0; i < n_incl; ++i) {
            const InclDev &q = incl[i];
            double f;
            if (q.shape == 0) {
                f = q.h[0] * sinc_pi(q.h[0] * n1) * q.h[1] * sinc_pi(q.h[1] * n2);
                if (d == 3) f *= q.h[2] * sinc_pi(q.h[2] * n3);
            } else {
                const double kn = sqrt((double)n1 * n1 + (double)n2 * n2);
                const double r = q.h[0];
                f = kn == 0.0 ? M_PI * r * r : r * j1(2.0 * M_PI * r * kn) / kn;
            }
            const double arg = -2.0 * ((double)n1 * q.c[0] + (double)n2 * q.c[1] + (d == 3 ? (double)n3 * q.c[2] : 0.0));
            double sv, cv;
            sincospi(arg, &sv, &cv);
            re += q.w * f * cv;
            im += q.w * f * sv;
        }
        out[idx] = make_double2(re, im);
    }
}


// ---------------------------------------------------------------------------
// Specialised transforms for the grid sizes in kFastSched: compile-time
// schedules with composite radices done in registers (Cooley-Tukey with
// constant internal twiddles), in-place stages staged through registers (one
// LDS buffer), and all d components of a batch transformed together.
// ---------------------------------------------------------------------------
// One in-place Stockham stage over NB transforms of length N: every thread
// first loads all inputs of its butterflies into registers, then (after a
// barrier) twiddles, transforms and stores them.  Column layout (ROWL false)
// with NA < NB: only the NA transforms 0 .. (NA - 1) / 2 and NB - NA / 2 ..
// NB - 1 (the non-zero frequencies of a zero-padded axis) are done.
template <typename T, int R, int N, int P, int NB, bool ROWL, int NT = kThreads, int NA = NB>
__device__ __forceinline__ void stage_ip(Vt<T> *X, const Vt<T> *__restrict__ tw, T sg) {
    constexpr int TQ = N / R;
    constexpr int NT_ = ROWL ? NB : NA;  // transforms done
    constexpr int TOT = TQ * NT_;
    constexpr int PER = (TOT + NT - 1) / NT;
    auto colmap = [](int c) { return c < (NA + 1) / 2 ? c : c + (NB - NA); };
    Vt<T> u[PER][R];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int idx = threadIdx.x + t * NT;
        if (PER * NT == TOT || idx < TOT) {
            const int b = ROWL ? idx / TQ : colmap(idx % NA);
            const int i = ROWL ? idx % TQ : idx / NA;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int pos = i + q * TQ;
                u[t][q] = ROWL ? X[b * N + pos] : X[pos * NB + b];
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int idx = threadIdx.x + t * NT;
        if (PER * NT == TOT || idx < TOT) {
            const int b = ROWL ? idx / TQ : colmap(idx % NA);
            const int i = ROWL ? idx % TQ : idx / NA;
            const int k = i % P;
            if constexpr (P > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    Vt<T> w = tw[(q - 1) * P + k];
                    w.y *= -sg;
                    u[t][q] = cmul(u[t][q], w);
                }
            }
            dftn<T, R>(u[t], sg);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int pos = j + q * P;
                if (ROWL)
                    X[b * N + pos] = u[t][q];
                else
                    X[pos * NB + b] = u[t][q];
            }
        }
    }
    __syncthreads();
}

template <typename T, int FI, int S, int P, int OFF, int NB, bool ROWL, int NT = kThreads, int NA = NB>
__device__ __forceinline__ void fft_ip(Vt<T> *X, const Vt<T> *tw, T sg) {
    if constexpr (S < kFastSched[FI].nst) {
        constexpr int R = kFastSched[FI].r[S];
        stage_ip<T, R, kFastSched[FI].n, P, NB, ROWL, NT, NA>(X, tw + OFF, sg);
        fft_ip<T, FI, S + 1, P * R, OFF + (R - 1) * P, NB, ROWL, NT, NA>(X, tw, sg);
    }
}


// Copy the n - 1 twiddles of a specialised transform into LDS (read by every
// stage; a global read per butterfly twiddle would stall each stage).
// Only short tables are staged: for n = 2025 the table (32 KB in FP64) would
// cost more occupancy than its reads cost latency.
constexpr bool tw_in_lds(int n, int es) { return n * es <= 12 * 1024; }
constexpr size_t tw_lds_entries(int n, int es) { return tw_in_lds(n, es) ? (size_t)n : 0; }
template <typename T, int N, int NTH = kThreads>
__device__ __forceinline__ const Vt<T> *twiddles_to_lds(Vt<T> *dst, const Vt<T> *__restrict__ src) {
    if constexpr (!tw_in_lds(N, sizeof(Vt<T>))) {
        return src;
    } else {
        for (int i = threadIdx.x; i < N - 1; i += NTH) dst[i] = src[i];
        return dst;
    }
}

// row pairs per work-group of the specialised anisotropic row pass so that
// one batch of all d components stays within 24 KB of LDS (the passes are
// latency-bound: smaller work-groups put more of them on a CU)
constexpr int fast_batch(int n, int es, int d) {
    const int cap = 24 * 1024;
    int b = 16;
    while (b > 1 && d * b * n * es > cap) b /= 2;
    return b;
}

// pencils per work-group of the specialised strided-axis pass: one batch of
// all d components within 24 KB of LDS, or 48 KB for 3D FP64 transforms of
// more than 225 points, where the larger batch keeps more of the work-group
// busy in the butterfly stages; elsewhere (2D, shorter 3D transforms) the
// smaller work-groups, more of them per CU, measured faster.  The 3D
// transforms of 225 points (order 113) take tiles sized to the rounds of
// resident work-groups, set by the axis-1 passes and their 113 x 57 pencils:
// in FP32, 9 pencils (50 KB of LDS, three work-groups per CU) make 716
// tiles, one round of the 768 work-groups that fit at once; in FP64 (twice
// the bytes, more than all LDS of the chip holds) 7 pencils (79 KB, two per
// CU) make 921 tiles, under two rounds of 512.  The 2D FP32 transforms of 729
// points (order 365) take 3 pencils with 512 threads (486 of the 2 x 3 x 81
// radix-9 butterflies busy in one round, against two rounds for 2 pencils and
// 256 threads): a batch of 16 such solves 7 % faster.
constexpr int pencil_batch(int n, int es, int d) {
    if (d == 3 && n == 225) return es >= 16 ? 7 : 9;
    if (es < 16 && d == 2 && n == 729) return 3;
    const int cap = (es >= 16 && d == 3 && n > 225) ? 48 * 1024 : 24 * 1024;
    int b = 16;
    while (b > 1 && d * b * n * es > cap) b /= 2;
    return b;
}

// Problem owning this work-group in a multi-problem launch (binary search of
// the work-group offsets); *lb receives the problem-local work-group index.
// Work-groups are dispatched to the 8 XCDs round-robin (physical index mod 8);
// each XCD has its own L2.  Map the physical index to a logical one so that
// every XCD receives a contiguous range of logical tiles: neighbouring tiles
// (which share 128-byte lines of the strided operands) then meet in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_logical(int b, int total) {
    const int q = total / kXcds, r = total % kXcds;
    const int x = b % kXcds, k = b / kXcds;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ int find_problem(const int *__restrict__ woff, int np, int *lb) {
    int lo = 0, hi = np - 1;
    const int bx = xcd_logical(blockIdx.x, gridDim.x);
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (woff[mid] <= bx)
            lo = mid;
        else
            hi = mid - 1;
    }
    *lb = bx - woff[lo];
    return lo;
}

// threads of the specialised strided-axis pass: 512 for the 2D FP64 pencils
// of 2025 points (one pencil of both components per work-group), the 2D FP32
// tiles of 729 points and the 3D tiles of 225 points (315 or 405 transforms of
// 15 points per stage), so that every stage of the transform takes one round
// of the threads; else 256
constexpr int pencil_nt(int n, int es, int d) {
    return ((es >= 16 && d == 2 && n >= 2025) || (es < 16 && d == 2 && n == 729) || (d == 3 && n == 225))
               ? 512
               : kThreads;
}

template <typename T, int FI, int D>
__global__ __launch_bounds__(pencil_nt(kFastSched[FI].n, sizeof(Vt<T>), D))
void pencil_fast(const PencilArgs *__restrict__ pa, const int *__restrict__ woff, int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int NT = pencil_nt(N, sizeof(V), D);
    constexpr int B = pencil_batch(N, sizeof(V), D);
    constexpr int NB = D * B;  // LDS layout [pos][component][batch]
    constexpr int LPI = NT / NB;  // positions per step of the plain prologue / epilogue
    int lb;
    const PencilArgs &a = pa[find_problem(woff, np, &lb)];
    if (a.status != nullptr && a.status->done) return;
    // loads of a starting work-group before the stages of running ones (the
    // priority drops again once the batch is in LDS)
    __builtin_amdgcn_s_setprio(3);
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    V *X = reinterpret_cast<V *>(smem_raw);
    const int gx = (a.nb + B - 1) / B;
    const int o = lb / gx;
    const int b0 = (lb - o * gx) * B;
    const int nbw = min(B, a.nb - b0);
    const V *tw = twiddles_to_lds<T, N, NT>(X + N * NB, reinterpret_cast<const V *>(a.tw) + a.f.twoff[0]);
    const T sg = T(a.sgn);
    const T scale = T(a.scale);
    const V zero = mk<T>(T(0), T(0));
    // pencil b0 + bb sits at (b0 + bb) / Nh, (b0 + bb) % Nh: one division per
    // work-group, then at most one carry per pencil (B <= Nh is not assumed)
    const int q0 = b0 / a.Nh, r0 = b0 - q0 * a.Nh;
    auto split = [&](int bb, int *qb, int *rb) {
        int r = r0 + bb, q = q0;
        while (r >= a.Nh) {
            r -= a.Nh;
            ++q;
        }
        *qb = q;
        *rb = r;
    };
    auto freq = [&](int l, int L, int bb, int *k1, int *k2, int *k3) {
        *k1 = wrapi(l, L);
        int qb, rb;
        split(bb, &qb, &rb);
        if (D == 3) {
            *k2 = wrapi(qb, a.Nmid);
            *k3 = rb;
        } else {
            *k2 = rb;
            *k3 = 0;
        }
    };
    // Global loads of a phase are issued together (branch-free, with idle
    // slots reading an in-range address) into scalar register arrays, then
    // written to LDS.  The input frequencies k in [-(L_in / 2), khi) sit at
    // positions 0 .. khi - 1 and N - L_in / 2 .. N - 1, so the positions
    // khi .. khi + N - L_in - 1 form one contiguous zero band of the LDS batch,
    // written by a loop of its own; slots of idle pencils in the input range
    // are written as zeros by the loading threads.  The trip counts are
    // compile-time bounds: inputs of at most (N + 1) / 2 points (zero-padded
    // transforms) or of N points.
    const int khi = (a.L_in + 1) / 2;
    if (a.pro == PRO_EXPAND) {
      // the CG vectors hold at most (N + 1) / 2 frequencies per axis (Ga), or N
      // (GaNi, transforms on the grid of the approximation order itself)
      auto expand = [&](auto cap) {
        constexpr int PE = (decltype(cap)::value * B + NT - 1) / NT;
        const auto *sr = gbl(reinterpret_cast<const V *>(a.st_r));
        auto *sp = gbl(reinterpret_cast<V *>(a.st_p));
        const auto *sx = gbl(reinterpret_cast<const V *>(a.st_x));
        const T beta = (a.update_p && a.status) ? T(a.status->beta) : T(0);
        T ax[PE][2], ay[PE][2], bx[PE][2], by[PE][2];
#pragma unroll
        for (int t = 0; t < PE; ++t) {
            const int idx = threadIdx.x + t * NT;
            const int bb = idx % B;
            const int l = idx / B;
            const bool ok = idx < a.L_in * B && bb < nbw;
            const long off = ok ? (long)l * a.in_ls + b0 + bb : (long)b0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const long o2 = (c < a.nc ? c : 0) * a.st_cs + off;
                const V va = a.update_p ? gld(sr + o2) : gld(sx + o2);
                const V vb = a.update_p ? gld(sp + o2) : zero;
                ax[t][c] = va.x;
                ay[t][c] = va.y;
                bx[t][c] = vb.x;
                by[t][c] = vb.y;
            }
        }
        for (int idx = threadIdx.x; idx < (N - a.L_in) * NB; idx += NT) X[khi * NB + idx] = zero;
#pragma unroll
        for (int t = 0; t < PE; ++t) {
            const int idx = threadIdx.x + t * NT;
            const int bb = idx % B;
            const int l = idx / B;
            if (idx >= a.L_in * B) continue;
            if (bb >= nbw) {  // idle pencil of a ragged tile
                const int pos = posmod(wrapi(l, a.L_in), N);
#pragma unroll
                for (int al = 0; al < D; ++al) X[pos * NB + al * B + bb] = zero;
                continue;
            }
            int k1, k2, k3;
            freq(l, a.L_in, bb, &k1, &k2, &k3);
            T tb[2][3];
            const int nt = basis<T>(D, a.kind, k1, k2, k3, tb);
            V v[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                v[c] = zero;
                if (c < a.nc) {
                    if (a.update_p) {
                        v[c] = mk<T>(ax[t][c] + beta * bx[t][c], ay[t][c] + beta * by[t][c]);
                        gst(sp + c * a.st_cs + (long)l * a.in_ls + b0 + bb, v[c]);
                    } else {
                        v[c] = mk<T>(ax[t][c], ay[t][c]);
                    }
                }
            }
            const int pos = posmod(k1, N);
            double pc = 1.0, ps = 0.0;
            if (has_shift(a)) shift_phase(a, k1, k2, k3, &pc, &ps);
#pragma unroll
            for (int al = 0; al < D; ++al) {
                T ex = T(0), ey = T(0);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    if (c < nt) {
                        ex -= tb[c][al] * v[c].y;
                        ey += tb[c][al] * v[c].x;
                    }
                }
                if (has_shift(a)) {
                    const T nx = ex * T(pc) - ey * T(ps);
                    ey = ex * T(ps) + ey * T(pc);
                    ex = nx;
                }
                X[pos * NB + al * B + bb] = mk<T>(ex, ey);
            }
        }
      };
      if (2 * a.L_in <= N + 1)
          expand(std::integral_constant<int, (N + 1) / 2>{});
      else
          expand(std::integral_constant<int, N>{});
    } else {
        // every thread owns one LDS slot rr (component c, pencil bb) of LPI
        // positions per step, so its addresses advance by a constant stride;
        // slots of idle pencils in the input range are written as zeros, the
        // zero band outside it by a loop over the band alone
        const int rr = threadIdx.x % NB;
        const int l0 = threadIdx.x / NB;
        const bool act = threadIdx.x < LPI * NB;
        const int c = rr / B;
        const int bb = rr - c * B;
        const auto *in = gbl(reinterpret_cast<const V *>(a.in) + (long)o * a.in_os + b0 + (long)c * a.in_cs + bb);
        auto load = [&](auto cap) {
            constexpr int P = (decltype(cap)::value + LPI - 1) / LPI;
            T vx[P], vy[P];
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const int l = l0 + t * LPI;
                const bool ok = act && l < a.L_in && bb < nbw;
                const V v = gld(in + (ok ? (long)l * a.in_ls : 0L));
                vx[t] = ok ? v.x : T(0);
                vy[t] = ok ? v.y : T(0);
            }
            const int nz = N - a.L_in;  // zero band: positions khi .. khi + nz - 1
            for (int l = l0; act && l < nz; l += LPI) X[(khi + l) * NB + rr] = zero;
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const int l = l0 + t * LPI;
                if (act && l < a.L_in) X[posmod(wrapi(l, a.L_in), N) * NB + rr] = mk<T>(vx[t], vy[t]);
            }
        };
        if (2 * a.L_in <= N + 1)
            load(std::integral_constant<int, (N + 1) / 2>{});
        else
            load(std::integral_constant<int, N>{});
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    fft_ip<T, FI, 0, 1, 0, NB, false, NT>(X, tw, sg);
    auto *out = gbl(reinterpret_cast<V *>(a.out));
    if (a.epi == EPI_PROJECT) {
      // the projected vector holds at most (N + 1) / 2 frequencies per axis (Ga) or N (GaNi)
      auto project = [&](auto cap) -> double {
        constexpr int PE = (decltype(cap)::value * B + NT - 1) / NT;
        const auto *dv = gbl(reinterpret_cast<const V *>(a.st_dot));
        T dx[PE][2], dy[PE][2];
        if (a.st_dot != nullptr) {
#pragma unroll
            for (int t = 0; t < PE; ++t) {
                const int idx = threadIdx.x + t * NT;
                const int bb = idx % B;
                const int l = idx / B;
                const bool ok = idx < a.L_out * B && bb < nbw;
                const long off = ok ? (long)l * a.out_ls + b0 + bb : (long)b0;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const V v = gld(dv + (c < a.nc ? c : 0) * a.out_cs + off);
                    dx[t][c] = v.x;
                    dy[t][c] = v.y;
                }
            }
        }
        double part = 0.0;
#pragma unroll
        for (int t = 0; t < PE; ++t) {
            const int idx = threadIdx.x + t * NT;
            const int bb = idx % B;
            const int l = idx / B;
            if (idx >= a.L_out * B || bb >= nbw) continue;
            int k1, k2, k3;
            freq(l, a.L_out, bb, &k1, &k2, &k3);
            T tb[2][3];
            const int nt = basis<T>(D, a.kind, k1, k2, k3, tb);
            const int pos = posmod(k1, N);
            V y[D];
#pragma unroll
            for (int al = 0; al < D; ++al) y[al] = X[pos * NB + al * B + bb];
            const double w = (D == 3 ? k3 : k2) == 0 ? 1.0 : 2.0;  // half spectrum: k_d > 0 counts twice
            double pc = 1.0, ps = 0.0;
            if (has_shift(a)) shift_phase(a, k1, k2, k3, &pc, &ps);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (c < a.nc) {
                    T qx = T(0), qy = T(0);
                    if (c < nt) {
#pragma unroll
                        for (int al = 0; al < D; ++al) {
                            const T tt = tb[c][al] * scale;
                            qx += tt * y[al].y;
                            qy -= tt * y[al].x;
                        }
                    }
                    const long off = c * a.out_cs + (long)l * a.out_ls + b0 + bb;
                    if (has_shift(a)) {  // S*(s): the conjugate phase
                        const T nx = qx * T(pc) + qy * T(ps);
                        qy = qy * T(pc) - qx * T(ps);
                        qx = nx;
                    }
                    if (a.accumulate) {
                        const V old = gld(out + off);
                        qx += old.x;
                        qy += old.y;
                    }
                    gst(out + off, mk<T>(qx, qy));
                    if (a.st_dot != nullptr) {
                        part += w * ((double)dx[t][c] * (double)qx + (double)dy[t][c] * (double)qy);
                    } else {
                        part += w * ((double)qx * (double)qx + (double)qy * (double)qy);
                    }
                }
            }
        }
        return part;
      };
      const double part = (2 * a.L_out <= N + 1) ? project(std::integral_constant<int, (N + 1) / 2>{})
                                                 : project(std::integral_constant<int, N>{});
        const double s = block_sum_t<NT>(part);
        if (threadIdx.x == 0) a.partial[lb] = s;
    } else {
        const int rr = threadIdx.x % NB;
        const int c = rr / B;
        const int bb = rr - c * B;
        if (threadIdx.x < LPI * NB && bb < nbw) {
            auto *ob = out + (long)c * a.out_cs + (long)o * a.out_os + b0 + bb;
            for (int l = threadIdx.x / NB; l < a.L_out; l += LPI) {
                V v = X[posmod(wrapi(l, a.L_out), N) * NB + rr];
                v.x *= scale;
                v.y *= scale;
                gst(ob + (long)l * a.out_ls, v);
            }
        }
    }
}

template <typename T, int FI, int D>
__global__ __launch_bounds__(kThreads) void row_fast(const RowArgs *__restrict__ ra, const int *__restrict__ woff,
                                                     int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int RP = fast_batch(N, sizeof(V), D);
    constexpr int NB = D * RP;  // LDS layout [component][row pair][pos]
    int lb;
    const RowArgs &a = ra[find_problem(woff, np, &lb)];
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    V *X = reinterpret_cast<V *>(smem_raw);
    const int nh = a.Nh_row;
    const V *tw = twiddles_to_lds<T, N>(X + N * NB, reinterpret_cast<const V *>(a.tw) + a.f.twoff[0]);
    V *data = reinterpret_cast<V *>(a.data);
    const T *g = reinterpret_cast<const T *>(a.g);
    const int pair0 = lb * RP;
    const int nvp = min(RP, (a.nrows + 1) / 2 - pair0);
    const V zero = mk<T>(T(0), T(0));
    T A0[D * D], Dm[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) {
        A0[i] = T(a.A0[i]);
        Dm[i] = T(a.D[i]);
    }
    // material values of this thread's grid points, loaded before the
    // transforms so that their latency overlaps them
    constexpr int MP = (RP * N + kThreads - 1) / kThreads;
    T gv1[MP], gv2[MP];
#pragma unroll
    for (int t = 0; t < MP; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        const int j = idx / N;
        const int x = idx - j * N;
        gv1[t] = T(0);
        gv2[t] = T(0);
        if (idx < RP * N && j < nvp && a.nfield <= 1) {
            const int r1 = 2 * (pair0 + j);
            gv1[t] = g[(long)r1 * N + x];
            if (r1 + 1 < a.nrows) gv2[t] = g[(long)(r1 + 1) * N + x];
        }
    }
    if (a.mode == ROW_OPER) {
        // both rows of every pair, all loads in flight together (nh <= (N + 1) / 2),
        // then the packed Hermitian extension; the zero band nh <= x <= N - nh
        // is written by a disjoint loop
        constexpr int PLR = (NB * ((N + 1) / 2) + kThreads - 1) / kThreads;
        const auto *dg = gbl(reinterpret_cast<const V *>(a.data));
        T p1x[PLR], p1y[PLR], p2x[PLR], p2y[PLR];
#pragma unroll
        for (int t = 0; t < PLR; ++t) {
            const int idx = threadIdx.x + t * kThreads;
            const int pc = idx / nh;
            const int kx = idx - pc * nh;
            const int c = pc / RP;
            const int j = pc - c * RP;
            const int r1 = 2 * (pair0 + j);
            const bool ok = idx < NB * nh && j < nvp;
            const bool ok2 = ok && r1 + 1 < a.nrows;
            const long off = ok ? (long)c * a.cs + (long)r1 * nh + kx : 0L;
            const V u1 = gld(dg + off);
            const V u2 = gld(dg + (ok2 ? off + nh : off));
            p1x[t] = u1.x;
            p1y[t] = u1.y;
            p2x[t] = ok2 ? u2.x : T(0);
            p2y[t] = ok2 ? u2.y : T(0);
        }
        for (int idx = threadIdx.x; idx < NB * (N - 2 * nh + 1); idx += kThreads) {
            const int pc = idx / (N - 2 * nh + 1);
            X[pc * N + nh + (idx - pc * (N - 2 * nh + 1))] = zero;
        }
#pragma unroll
        for (int t = 0; t < PLR; ++t) {
            const int idx = threadIdx.x + t * kThreads;
            const int pc = idx / nh;
            const int kx = idx - pc * nh;
            if (idx >= NB * nh) continue;
            const V u1 = mk<T>(p1x[t], p1y[t]);
            const V u2 = mk<T>(p2x[t], p2y[t]);
            if (kx == 0) {
                X[pc * N] = mk<T>(u1.x, u2.x);
            } else {
                X[pc * N + kx] = mk<T>(u1.x - u2.y, u1.y + u2.x);
                X[pc * N + N - kx] = mk<T>(u1.x + u2.y, u2.x - u1.y);
            }
        }
        __syncthreads();
        fft_ip<T, FI, 0, 1, 0, NB, true>(X, tw, T(1));
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const int idx = threadIdx.x + t * kThreads;
            const int j = idx / N;
            const int x = idx - j * N;
            if (idx >= RP * N || j >= nvp) continue;
            V e[D];
#pragma unroll
            for (int b = 0; b < D; ++b) e[b] = X[(b * RP + j) * N + x];
            T m1[D * D], m2[D * D];
            if (a.nfield > 1) {
                const int r1 = 2 * (pair0 + j);
                sym_load<T>(g, a.gstride, (long)r1 * N + x, D, m1);
                if (r1 + 1 < a.nrows)
                    sym_load<T>(g, a.gstride, (long)(r1 + 1) * N + x, D, m2);
                else
#pragma unroll
                    for (int i = 0; i < D * D; ++i) m2[i] = T(0);
            } else {
                const T g1 = gv1[t];
                const T g2 = gv2[t];
#pragma unroll
                for (int i = 0; i < D * D; ++i) {
                    m1[i] = A0[i] + g1 * Dm[i];
                    m2[i] = A0[i] + g2 * Dm[i];
                }
            }
#pragma unroll
            for (int al = 0; al < D; ++al) {
                T y1 = T(0), y2 = T(0);
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    y1 += m1[al * D + b] * e[b].x;
                    y2 += m2[al * D + b] * e[b].y;
                }
                X[(al * RP + j) * N + x] = mk<T>(y1, y2);
            }
        }
    } else {  // ROW_RHS: y = A(x) E on both rows, |y|^2 and y.E partial sums
        double load = 0.0, work = 0.0;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const int idx = threadIdx.x + t * kThreads;
            if (idx >= RP * N) continue;
            const int j = idx / N;
            const int x = idx - j * N;
            V y[D];
#pragma unroll
            for (int al = 0; al < D; ++al) y[al] = zero;
            if (j < nvp) {
                const int r1 = 2 * (pair0 + j);
                const int r2 = r1 + 1;
                const bool v2 = r2 < a.nrows;
                T m1[D * D], m2[D * D];
                if (a.nfield > 1) {
                    sym_load<T>(g, a.gstride, (long)r1 * N + x, D, m1);
                    if (v2)
                        sym_load<T>(g, a.gstride, (long)r2 * N + x, D, m2);
                    else
#pragma unroll
                        for (int i = 0; i < D * D; ++i) m2[i] = T(0);
                } else {
                    const T g1 = gv1[t];
                    const T g2 = gv2[t];
#pragma unroll
                    for (int i = 0; i < D * D; ++i) {
                        m1[i] = A0[i] + g1 * Dm[i];
                        m2[i] = A0[i] + g2 * Dm[i];
                    }
                }
#pragma unroll
                for (int al = 0; al < D; ++al) {
                    T y1 = T(0), y2 = T(0);
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        y1 += m1[al * D + b] * T(a.E[b]);
                        if (v2) y2 += m2[al * D + b] * T(a.E[b]);
                    }
                    y[al] = mk<T>(y1, y2);
                    load += (double)y1 * y1 + (double)y2 * y2;
                    work += ((double)y1 + (double)y2) * a.E[al];
                }
            }
#pragma unroll
            for (int al = 0; al < D; ++al) X[(al * RP + j) * N + x] = y[al];
        }
        const double s = block_sum(load);
        const double s2 = block_sum(work);
        if (threadIdx.x == 0) {
            a.partial[lb] = s;
            if (a.partial2 != nullptr) a.partial2[lb] = s2;
        }
    }
    __syncthreads();
    fft_ip<T, FI, 0, 1, 0, NB, true>(X, tw, T(-1));
    const T half = T(a.scale) * T(0.5);
    for (int idx = threadIdx.x; idx < NB * nh; idx += kThreads) {
        const int pc = idx / nh;
        const int kx = idx - pc * nh;
        const int c = pc / RP;
        const int j = pc - c * RP;
        if (j >= nvp) continue;
        const int r1 = 2 * (pair0 + j);
        const int r2 = r1 + 1;
        const V w = X[pc * N + kx];
        const V wm = X[pc * N + (kx == 0 ? 0 : N - kx)];
        data[(long)c * a.cs + (long)r1 * nh + kx] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
        if (r2 < a.nrows)
            data[(long)c * a.cs + (long)r2 * nh + kx] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
    }
}


// ---------------------------------------------------------------------------
// Operator row pass for isotropic materials, A(x) = (a0 + g(x) dA) I.  Every
// component row is multiplied by the same scalar field, so each packed row
// pair (two real rows as one complex transform) is independent of the others.
// The first inverse stage reads its points straight from the half-spectrum
// rows (Hermitian extension and zero padding on the fly); the last inverse
// stage leaves each thread holding the points x = i + q N/R, where the
// material multiply is applied and the first forward stage (same radix, same
// points) follows in registers.  Only the middle stages, the exchanges
// between stages and the final Hermitian unpacking go through LDS.
constexpr bool palindromic(int fi) {
    const int s = kFastSched[fi].nst;
    for (int i = 0; i < s; ++i)
        if (kFastSched[fi].r[i] != kFastSched[fi].r[s - 1 - i]) return false;
    return true;
}
constexpr int sched_p(int fi, int st) {
    int p = 1;
    for (int i = 0; i < st; ++i) p *= kFastSched[fi].r[i];
    return p;
}
constexpr int sched_off(int fi, int st) {
    int off = 0, p = 1;
    for (int i = 0; i < st; ++i) {
        off += (kFastSched[fi].r[i] - 1) * p;
        p *= kFastSched[fi].r[i];
    }
    return off;
}
// transforms per work-group and work-group size: every thread of the first
// and last stages owns one butterfly of radix r[0]
constexpr int iso_tb(int fi) {
    const int tq = kFastSched[fi].n / kFastSched[fi].r[0];
    // transforms of more than 128 butterflies per stage (n = 2025): one per
    // work-group, so that several share a CU
    return tq <= 64 ? 128 / tq : (tq <= 128 ? 256 / tq : 1);
}
constexpr int iso_nt(int fi) {
    const int tq = kFastSched[fi].n / kFastSched[fi].r[0];
    return (iso_tb(fi) * tq + 63) / 64 * 64;
}

template <typename T, int FI, int S, int SEND, int NB, int NT>
__device__ __forceinline__ void fft_mid(Vt<T> *X, const Vt<T> *tw, T sg) {
    if constexpr (S < SEND) {
        stage_ip<T, kFastSched[FI].r[S], kFastSched[FI].n, sched_p(FI, S), NB, true, NT>(X, tw + sched_off(FI, S),
                                                                                          sg);
        fft_mid<T, FI, S + 1, SEND, NB, NT>(X, tw, sg);
    }
}

template <typename T, int FI>
__global__ __launch_bounds__(iso_nt(FI)) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 1)))
void row_iso_fast(const RowArgs *__restrict__ ra,
                                                           const int *__restrict__ woff, int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int S = kFastSched[FI].nst;
    constexpr int R = kFastSched[FI].r[0];
    constexpr int TQ = N / R;  // butterflies per transform in the first and last stages
    constexpr int TB = iso_tb(FI);
    constexpr int NT = iso_nt(FI);
    constexpr int OFFL = sched_off(FI, S - 1);  // twiddles of the last stage (P = TQ)
    static_assert(palindromic(FI) && S >= 2 && sched_p(FI, S - 1) == TQ, "schedule must be palindromic");
    int lb;
    const RowArgs &a = ra[find_problem(woff, np, &lb)];
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    V *X = reinterpret_cast<V *>(smem_raw);  // [transform][pos]
    // stage twiddles staged in LDS when short; for the longest rows (2025
    // points, 32 KB in FP64) the LDS goes to the transforms and the twiddles
    // are read through the cache
    const V *twg = reinterpret_cast<const V *>(a.tw) + a.f.twoff[0];
    const V *tws = twiddles_to_lds<T, N, NT>(X + TB * N, twg);
    const V zero = mk<T>(T(0), T(0));
    const int nh = a.Nh_row;
    const int npairs = (a.nrows + 1) / 2;
    const int ntr = a.d * npairs;
    const int tl = threadIdx.x / TQ;
    const int i = threadIdx.x - tl * TQ;
    const int tb = lb * TB + tl;
    const bool act = tl < TB && tb < ntr;
    // transforms ordered pair-major (components fastest), so that the d
    // transforms reading one row pair's material values share a work-group
    int c = 0, r1 = 0;
    if (act) {
        const int pr = tb / a.d;
        c = tb - pr * a.d;
        r1 = 2 * pr;
    }
    const bool v2 = act && r1 + 1 < a.nrows;
    const V *data = reinterpret_cast<const V *>(a.data);
    const V *row1 = data + (long)c * a.cs + (long)r1 * nh;
    const T *g = reinterpret_cast<const T *>(a.g);
    const T a0 = T(a.A0[0]);
    const T da = T(a.D[0]);
    V u[R];
    {
        // all loads first (idle points read entry 0 of the pair), then the
        // Hermitian packing by selects
        T l1x[R], l1y[R], l2x[R], l2y[R];
        const auto *rg = gbl(row1);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int pos = i + q * TQ;
            const int kx = pos < nh ? pos : (pos > N - nh ? N - pos : 0);
            const V a1 = gld(rg + kx);
            const V a2 = gld(rg + (v2 ? nh + kx : kx));
            l1x[q] = a1.x;
            l1y[q] = a1.y;
            l2x[q] = a2.x;
            l2y[q] = a2.y;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int pos = i + q * TQ;
            const V u1 = mk<T>(l1x[q], l1y[q]);
            const V u2 = v2 ? mk<T>(l2x[q], l2y[q]) : zero;
            const V lo = pos == 0 ? mk<T>(u1.x, u2.x) : mk<T>(u1.x - u2.y, u1.y + u2.x);
            const V hi = mk<T>(u1.x + u2.y, u2.x - u1.y);
            u[q] = !act ? zero : (pos < nh ? lo : (pos > N - nh ? hi : zero));
        }
    }
    // first inverse stage (P = 1): outputs at i R + q
    dftn<T, R>(u, T(1));
    if (act) {
#pragma unroll
        for (int q = 0; q < R; ++q) X[tl * N + i * R + q] = u[q];
    }
    __syncthreads();
    fft_mid<T, FI, 1, S - 1, TB, NT>(X, tws, T(1));
    // last inverse stage: inputs and outputs at i + q TQ (own points only)
    if (act) {
#pragma unroll
        for (int q = 0; q < R; ++q) u[q] = X[tl * N + i + q * TQ];
    }
    __syncthreads();
#pragma unroll
    for (int q = 1; q < R; ++q) {
        V w = tws[OFFL + (q - 1) * TQ + i];
        w.y = -w.y;
        u[q] = cmul(u[q], w);
    }
    dftn<T, R>(u, T(1));
    // the two real rows at x = i + q TQ: multiply by a0 + g da (the material
    // values are loaded here, not held through the inverse stages; idle lanes
    // read row r1, in range, and their products are never stored)
    {
        const T *gr1 = g + (long)r1 * N + i;
        const T *gr2 = v2 ? gr1 + N : gr1;
        T g1[R], g2[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            g1[q] = gr1[q * TQ];
            g2[q] = gr2[q * TQ];
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            u[q].x *= a0 + g1[q] * da;
            u[q].y *= a0 + g2[q] * da;
        }
    }
    // first forward stage on the same points
    dftn<T, R>(u, T(-1));
    if (act) {
#pragma unroll
        for (int q = 0; q < R; ++q) X[tl * N + i * R + q] = u[q];
    }
    __syncthreads();
    fft_mid<T, FI, 1, S - 1, TB, NT>(X, tws, T(-1));
    if (act) {
#pragma unroll
        for (int q = 0; q < R; ++q) u[q] = X[tl * N + i + q * TQ];
#pragma unroll
        for (int q = 1; q < R; ++q) u[q] = cmul(u[q], tws[OFFL + (q - 1) * TQ + i]);
        dftn<T, R>(u, T(-1));
#pragma unroll
        for (int q = 0; q < R; ++q) X[tl * N + i + q * TQ] = u[q];
    }
    __syncthreads();
    // unpack the two rows of each transform and keep the first nh frequencies
    V *out = reinterpret_cast<V *>(a.data);
    const T half = T(a.scale) * T(0.5);
    for (int o = threadIdx.x; o < TB * nh; o += NT) {
        const int t = o / nh;
        const int kx = o - t * nh;
        const int tbo = lb * TB + t;
        if (tbo >= ntr) continue;
        const int po = tbo / a.d;
        const int co = tbo - po * a.d;
        const int ro = 2 * po;
        const V w = X[t * N + kx];
        const V wm = X[t * N + (kx == 0 ? 0 : N - kx)];
        V *orow = out + (long)co * a.cs + (long)ro * nh;
        orow[kx] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
        if (ro + 1 < a.nrows) orow[nh + kx] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
    }
}

// Variant for two-stage schedules: every exchange between stages moves the
// real parts through LDS first and the imaginary parts second, so a transform
// needs n reals of LDS instead of n complex values; with the material values
// loaded at the multiply (not held in registers) this raises the resident
// waves, which hides the latencies of the stages, and each thread unpacks its
// own points (no index division).
constexpr int split_tb(int fi) { return iso_tb(fi); }
constexpr int split_nt(int fi) { return iso_nt(fi); }

template <typename T, int FI>
__global__ __launch_bounds__(split_nt(FI)) void row_iso_split(const RowArgs *__restrict__ ra,
                                                             const int *__restrict__ woff, int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int R = kFastSched[FI].r[0];
    constexpr int TQ = N / R;
    constexpr int TB = split_tb(FI);
    constexpr int NT = split_nt(FI);
    constexpr int OFFL = sched_off(FI, 1);
    static_assert(kFastSched[FI].nst == 2 && kFastSched[FI].r[1] == R, "two-stage palindromic schedule");
    int lb;
    const RowArgs &a = ra[find_problem(woff, np, &lb)];
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    T *Bf = reinterpret_cast<T *>(smem_raw);            // [transform][pos], one part at a time
    V *tws = reinterpret_cast<V *>(Bf + TB * N);        // last-stage twiddles
    const V *twg = reinterpret_cast<const V *>(a.tw) + a.f.twoff[0];
    for (int i = threadIdx.x; i < N - 1; i += NT) tws[i] = twg[i];
    const V zero = mk<T>(T(0), T(0));
    const int nh = a.Nh_row;
    const int npairs = (a.nrows + 1) / 2;
    const int ntr = a.d * npairs;
    const int tl = threadIdx.x / TQ;
    const int i = threadIdx.x - tl * TQ;
    const int tb = lb * TB + tl;
    const bool act = tl < TB && tb < ntr;
    int c = 0, r1 = 0;
    if (act) {
        const int pr = tb / a.d;
        c = tb - pr * a.d;
        r1 = 2 * pr;
    }
    const bool v2 = act && r1 + 1 < a.nrows;
    V *data = reinterpret_cast<V *>(a.data);
    V *row1 = data + (long)c * a.cs + (long)r1 * nh;
    V *row2 = row1 + nh;
    const T *g = reinterpret_cast<const T *>(a.g);
    T *Bt = Bf + (act ? tl : 0) * N;
    // exchange: write own values at positions wp(q), read positions rp(q)
    auto xchg = [&](V *u, auto wp, auto rp) {
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (act) Bt[wp(q)] = u[q].x;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (act) u[q].x = Bt[rp(q)];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (act) Bt[wp(q)] = u[q].y;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (act) u[q].y = Bt[rp(q)];
        __syncthreads();
    };
    auto stage_out = [&](int q) { return i * R + q; };
    auto own = [&](int q) { return i + q * TQ; };
    V u[R];
    {
        // loads in two groups (idle points read entry 0 of the pair), each
        // followed by the Hermitian packing by selects; the empty asm
        // statements keep the second group from being hoisted, which bounds
        // the registers the staged values need
        const auto *rg = gbl(row1);
        constexpr int LG = (R + 1) / 2;
#pragma unroll
        for (int q0 = 0; q0 < R; q0 += LG) {
            asm volatile("" ::: "memory");
            T l1x[LG], l1y[LG], l2x[LG], l2y[LG];
#pragma unroll
            for (int q = q0; q < q0 + LG && q < R; ++q) {
                const int pos = i + q * TQ;
                const int kx = pos < nh ? pos : (pos > N - nh ? N - pos : 0);
                const V a1 = gld(rg + kx);
                const V a2 = gld(rg + (v2 ? nh + kx : kx));
                l1x[q - q0] = a1.x;
                l1y[q - q0] = a1.y;
                l2x[q - q0] = a2.x;
                l2y[q - q0] = a2.y;
            }
#pragma unroll
            for (int q = q0; q < q0 + LG && q < R; ++q) {
                const int pos = i + q * TQ;
                const V u1 = mk<T>(l1x[q - q0], l1y[q - q0]);
                const V u2 = v2 ? mk<T>(l2x[q - q0], l2y[q - q0]) : zero;
                const V lo = pos == 0 ? mk<T>(u1.x, u2.x) : mk<T>(u1.x - u2.y, u1.y + u2.x);
                const V hi = mk<T>(u1.x + u2.y, u2.x - u1.y);
                u[q] = !act ? zero : (pos < nh ? lo : (pos > N - nh ? hi : zero));
            }
        }
        asm volatile("" ::: "memory");
    }
    dftn<T, R>(u, T(1));
    xchg(u, stage_out, own);
#pragma unroll
    for (int q = 1; q < R; ++q) {
        V w = tws[OFFL + (q - 1) * TQ + i];
        w.y = -w.y;
        u[q] = cmul(u[q], w);
    }
    dftn<T, R>(u, T(1));
    {
        // material values in groups of five loads, issued only here (the
        // empty asm statements keep the compiler from hoisting them over
        // the transform, where they would hold registers)
        const T a0 = T(a.A0[0]);
        const T da = T(a.D[0]);
        const T *g1 = g + (long)r1 * N + i;
        const T *g2 = v2 ? g1 + N : g1;
        constexpr int GQ = 5;
#pragma unroll
        for (int q0 = 0; q0 < R; q0 += GQ) {
            asm volatile("" ::: "memory");
#pragma unroll
            for (int q = q0; q < q0 + GQ && q < R; ++q) {
                const T ga = g1[q * TQ];
                const T gb = g2[q * TQ];
                u[q].x *= a0 + ga * da;
                u[q].y *= a0 + gb * da;
            }
        }
        asm volatile("" ::: "memory");
    }
    dftn<T, R>(u, T(-1));
    xchg(u, stage_out, own);
#pragma unroll
    for (int q = 1; q < R; ++q) u[q] = cmul(u[q], tws[OFFL + (q - 1) * TQ + i]);
    dftn<T, R>(u, T(-1));
    // Hermitian unpacking: each thread pairs its points p < nh with N - p
    // (nh <= (N + 1) / 2, so only the first QH of its points are kept)
    constexpr int QH = ((N + 1) / 2 + TQ - 1) / TQ;
    V m[QH];
    auto partner = [&](int q) {
        const int p = i + q * TQ;
        return p == 0 ? 0 : N - p;
    };
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (act) Bt[own(q)] = u[q].x;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q)
        if (act) m[q].x = Bt[partner(q)];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (act) Bt[own(q)] = u[q].y;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q)
        if (act) m[q].y = Bt[partner(q)];
    const T half = T(a.scale) * T(0.5);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int p = i + q * TQ;
        if (act && p < nh) {
            const V w = u[q];
            const V wm = m[q];
            row1[p] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
            if (v2) row2[p] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
        }
    }
}

// Variant for the row lengths of Ga plans (half-spectrum rows of at most
// (N + 3) / 4 points: order (N + 1) / 2 on the grid N).  Every global load of
// a work-group -- its half-spectrum rows, the material rows of its pairs and
// the last-stage twiddles -- is issued at once and parked in LDS, so a
// work-group waits for memory once.  Work-groups own whole row pairs (all D
// components of each, pair-major), so each material row is fetched once.
// Lanes beyond the last transform repeat the work of the last one, and the
// spare lane of a 16-lane group that of the group's 15th (same inputs, same
// instructions, so their LDS writes store the values already there) instead
// of branching around every LDS access; only the final stores are guarded.
// The transform is that of row_iso_split; per-transform LDS rows are padded
// so that the stride exchanges of neighbouring transforms fall into
// different banks.
constexpr int staged_nhc(int n) { return (n + 3) / 4; }
// lanes per transform: 15 butterflies get an aligned group of 16 lanes (the
// last lane repeats the 15th), so that the lanes of one LDS access pass belong
// to whole transforms
constexpr int staged_lg(int fi) {
    const int tq = kFastSched[fi].n / kFastSched[fi].r[0];
    return tq == 15 ? 16 : tq;
}
// threads per work-group: the best lane utilisation of 128, 192 or 256, except
// for the 3D FP64 rows of 225 points (es: bytes of a complex value), which
// take 256 (five row pairs, three work-groups per CU): 2 % faster than the
// 192 of the best utilisation, while in FP32 the two were alike
constexpr int staged_nt(int fi, int d, int es) {
    if (es >= 16 && d == 3 && kFastSched[fi].n == 225) return 256;
    const int tq = kFastSched[fi].n / kFastSched[fi].r[0];
    int best = 128, bu = 0;  // utilisation in 1/1024
    for (int nt = 128; nt <= 256; nt += 64) {
        const int tb = (nt / staged_lg(fi)) / d * d;
        const int u = tb * tq * 1024 / nt;
        if (u > bu) {
            bu = u;
            best = nt;
        }
    }
    return best;
}
constexpr int staged_tb(int fi, int d, int es) { return (staged_nt(fi, d, es) / staged_lg(fi)) / d * d; }
// LDS row stride of one transform (in reals): 240 = 16 (mod 32) for n = 225
constexpr int staged_stride(int fi) { return kFastSched[fi].n == 225 ? 240 : kFastSched[fi].n; }
// twiddles of the second stage: w_n^(q i) at (q - 1) n / r + i (1 <= q < r,
// 0 <= i < n / r), so that the lanes of a transform read consecutive entries
constexpr int staged_ntp(int fi) { return (kFastSched[fi].r[0] - 1) * (kFastSched[fi].n / kFastSched[fi].r[0]); }
template <typename T>
constexpr size_t staged_lds(int fi, int d) {
    const int n = kFastSched[fi].n, tb = staged_tb(fi, d, (int)sizeof(Vt<T>));
    const size_t work = std::max(sizeof(Vt<T>) * tb * 2 * (staged_nhc(n) + 1), sizeof(T) * tb * staged_stride(fi));
    const size_t gm = sizeof(T) * (tb / d) * 2 * n;
    return (gm + 15) / 16 * 16 + sizeof(Vt<T>) * staged_ntp(fi) + work;
}

// three waves per SIMD: what the LDS of four 192-thread or three 256-thread
// work-groups per CU allows in FP64
template <typename T, int FI, int D>
__global__ __launch_bounds__(staged_nt(FI, D, sizeof(Vt<T>))) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 1)))
void row_iso_staged(const RowArgs *__restrict__ ra,
                                                                  const int *__restrict__ woff, int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int R = kFastSched[FI].r[0];
    constexpr int TQ = N / R;
    constexpr int TB = staged_tb(FI, D, sizeof(Vt<T>));
    constexpr int PW = TB / D;  // row pairs per work-group
    constexpr int NT = staged_nt(FI, D, sizeof(Vt<T>));
    constexpr int NHC = staged_nhc(N);
    constexpr int SR = NHC + 1;  // staged row: NHC points and a zero slot
    constexpr int S = staged_stride(FI);
    constexpr int NTP = staged_ntp(FI);
    constexpr int OFFL = sched_off(FI, 1);
    constexpr int LG = staged_lg(FI);
    static_assert(kFastSched[FI].nst == 2 && kFastSched[FI].r[1] == R, "two-stage palindromic schedule");
    static_assert(TB * LG <= NT && TB % D == 0 && NT - TB * LG <= LG && LG >= TQ, "work-group shape");
    int lb;
    const RowArgs &a = ra[find_problem(woff, np, &lb)];
    if (a.status != nullptr && a.status->done) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    T *Gs = reinterpret_cast<T *>(smem_raw);                                           // [2 PW][N] material
    V *tp = reinterpret_cast<V *>(smem_raw + (sizeof(T) * PW * 2 * N + 15) / 16 * 16);  // [NTP] stage twiddles
    V *St = tp + NTP;                      // [D][2 PW][SR] staged half-spectrum rows ...
    T *Bf = reinterpret_cast<T *>(St);     // ... later [TB][S], one part at a time
    const int nh = a.Nh_row;
    const int npairs = (a.nrows + 1) / 2;
    const int pr0 = lb * PW;
    const int npr = min(PW, npairs - pr0);
    const int nrow_wg = min(2 * npr, a.nrows - 2 * pr0);  // rows of this work-group
    // ---- all global loads in flight together, then parked in LDS; the waves
    // of a work-group issuing its loads take priority over those already in
    // the transform arithmetic, so that a new work-group's loads leave early
    __builtin_amdgcn_s_setprio(3);
    constexpr int GP = (PW * 2 * N + NT - 1) / NT;
    constexpr int RS = 2 * PW * SR;  // staged slots of one component: its 2 PW rows
    constexpr int SPC = (RS + NT - 1) / NT;
    constexpr int NW = (R - 1) * TQ;  // stage-1 twiddles
    constexpr int WP = (NW + NT - 1) / NT;
    const auto *gsrc = gbl(reinterpret_cast<const T *>(a.g) + (long)2 * pr0 * N);
    const auto *dsrc = gbl(reinterpret_cast<const V *>(a.data));
    const auto *twg = gbl(reinterpret_cast<const V *>(a.tw) + a.f.twoff[0] + OFFL);
    const int gcnt = nrow_wg * N;
    T gv[GP];
    T sx[D][SPC], sy[D][SPC];
    T wx[WP], wy[WP];
#pragma unroll
    for (int t = 0; t < GP; ++t) {
        const int idx = threadIdx.x + t * NT;
        gv[t] = gsrc[idx < gcnt ? idx : 0];
    }
    // the rows of a work-group are contiguous in each component: one flat
    // copy per component into slots [c][row][SR] (slot k >= nh and rows past
    // the last are zero), with the offsets of a component in 32 bits
#pragma unroll
    for (int c = 0; c < D; ++c) {
        const auto *dc = dsrc + (long)c * a.cs + (long)2 * pr0 * nh;
#pragma unroll
        for (int t = 0; t < SPC; ++t) {
            const int f = threadIdx.x + t * NT;
            const int row = f / SR;
            const int k = f - row * SR;
            const bool ok = f < RS && k < nh && row < nrow_wg;
            const V v = gld(dc + (ok ? row * nh + k : 0));
            sx[c][t] = ok ? v.x : T(0);
            sy[c][t] = ok ? v.y : T(0);
        }
    }
#pragma unroll
    for (int t = 0; t < WP; ++t) {
        const int idx = threadIdx.x + t * NT;
        const V v = gld(twg + (idx < NW ? idx : 0));
        wx[t] = v.x;
        wy[t] = v.y;
    }
#pragma unroll
    for (int t = 0; t < GP; ++t) {
        const int idx = threadIdx.x + t * NT;
        if (idx < PW * 2 * N) Gs[idx] = idx < gcnt ? gv[t] : T(0);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) {
#pragma unroll
        for (int t = 0; t < SPC; ++t) {
            const int f = threadIdx.x + t * NT;
            if (f < RS) St[c * RS + f] = mk<T>(sx[c][t], sy[c][t]);
        }
    }
#pragma unroll
    for (int t = 0; t < WP; ++t) {
        const int idx = threadIdx.x + t * NT;
        if (idx < NW) tp[idx] = mk<T>(wx[t], wy[t]);
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    // ---- packed Hermitian extension of the two rows of this thread's transform
    const int tr = threadIdx.x / LG;
    const int lane = threadIdx.x - tr * LG;
    const int tl = tr < TB ? tr : TB - 1;  // lanes past the last transform repeat it
    const int i = lane < TQ ? lane : TQ - 1;  // and spare lanes of a group repeat its last
    const int lp = tl / D;                 // pair within the work-group
    const int c = tl - lp * D;             // component
    const bool owner = tr < TB && lane < TQ && lp < npr;
    // Points i + q TQ of this thread that lie in the zero band for every
    // thread (NHC <= q TQ and q TQ + TQ - 1 <= N - NHC) are zero on input and
    // not needed on output: with the band known at compile time the compiler
    // drops their arithmetic from the first inverse and the last forward stage.
    auto zband = [](int q) { return q * TQ >= NHC && q * TQ + TQ - 1 <= N - NHC; };
    V u[R];
    {
        const V *s1 = St + c * RS + 2 * lp * SR;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            if (zband(q)) {
                u[q] = mk<T>(T(0), T(0));
                continue;
            }
            // z = u1 + i u2 at p < nh, conj(u1) + i conj(u2) at p > N - nh,
            // (u1.x, u2.x) at p = 0, zero between (the zero slot)
            const int pos = i + q * TQ;
            const bool low = pos < nh;
            const int kx = low ? pos : (pos > N - nh ? N - pos : NHC);
            const V u1 = s1[kx];
            const V u2 = s1[SR + kx];
            const T sg = low ? (pos == 0 ? T(0) : T(1)) : T(-1);
            u[q] = mk<T>(u1.x - sg * u2.y, u2.x + sg * u1.y);
        }
    }
    __syncthreads();  // St is reused as Bf
    T *Bt = Bf + tl * S;
    auto xchg = [&](V *w, auto wp, auto rp) {
#pragma unroll
        for (int q = 0; q < R; ++q) Bt[wp(q)] = w[q].x;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q) w[q].x = Bt[rp(q)];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q) Bt[wp(q)] = w[q].y;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < R; ++q) w[q].y = Bt[rp(q)];
        __syncthreads();
    };
    auto stage_out = [&](int q) { return i * R + q; };
    auto own = [&](int q) { return i + q * TQ; };
    dftn<T, R>(u, T(1));
    xchg(u, stage_out, own);
#pragma unroll
    for (int q = 1; q < R; ++q) {
        V w = tp[(q - 1) * TQ + i];
        w.y = -w.y;
        u[q] = cmul(u[q], w);
    }
    dftn<T, R>(u, T(1));
    {
        const T a0 = T(a.A0[0]);
        const T da = T(a.D[0]);
        const T *g1 = Gs + 2 * lp * N + i;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            u[q].x *= a0 + g1[q * TQ] * da;
            u[q].y *= a0 + g1[N + q * TQ] * da;
        }
    }
    dftn<T, R>(u, T(-1));
    xchg(u, stage_out, own);
#pragma unroll
    for (int q = 1; q < R; ++q) u[q] = cmul(u[q], tp[(q - 1) * TQ + i]);
    dftn<T, R>(u, T(-1));
    // Hermitian unpacking: outputs p < nh <= NHC pair with N - p > N - NHC,
    // so only the points that can lie there go through LDS
    constexpr int QH = (NHC + TQ - 1) / TQ;
    V m[QH];
    auto partner = [&](int q) {
        const int p = i + q * TQ;
        return p == 0 ? 0 : N - p;
    };
    auto high = [](int q) { return q * TQ + TQ - 1 > N - NHC; };
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (high(q)) Bt[own(q)] = u[q].x;
    Bt[own(0)] = u[0].x;  // p = 0 pairs with itself
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q) m[q].x = Bt[partner(q)];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (high(q)) Bt[own(q)] = u[q].y;
    Bt[own(0)] = u[0].y;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QH; ++q) m[q].y = Bt[partner(q)];
    if (!owner) return;
    const int r1 = 2 * (pr0 + lp);
    const bool v2 = 2 * lp + 1 < nrow_wg;
    auto *row1 = gbl(reinterpret_cast<V *>(a.data) + (long)c * a.cs + (long)r1 * nh);
    const T half = T(a.scale) * T(0.5);
#pragma unroll
    for (int q = 0; q < QH; ++q) {
        const int p = i + q * TQ;
        if (p < nh) {
            const V w = u[q];
            const V wm = m[q];
            gst(row1 + p, mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half));
            if (v2) gst(row1 + nh + p, mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half));
        }
    }
}

// Launch target of the specialised kernels: the stream and, for timing, the
// events the dispatch records at its own start and end.
struct Disp {
    hipStream_t s;
    LaunchEv ev;
    Disp(hipStream_t st, LaunchEv e = LaunchEv{}) : s(st), ev(e) {}
};
template <typename... KArgs, typename... Args>
void dispatch(void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds, const Disp &d, Args... args) {
    if (d.ev.start != nullptr)
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, d.s, d.ev.start, d.ev.stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds, d.s, args...);
}

template <typename T, int FI, int D>
void launch_pencil_fast_t(const PencilArgs *args, const int *woff, int np, int total, const Disp &s) {
    constexpr int N = kFastSched[FI].n;
    constexpr int B = pencil_batch(N, sizeof(Vt<T>), D);
    const size_t lds = sizeof(Vt<T>) * ((size_t)N * D * B + tw_lds_entries(N, sizeof(Vt<T>)));
    dispatch((pencil_fast<T, FI, D>), dim3(total), dim3(pencil_nt(N, sizeof(Vt<T>), D)), lds, s, args, woff, np);
}

template <typename T, int FI, int D>
void launch_row_fast_t(const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    constexpr int N = kFastSched[FI].n;
    constexpr int RP = fast_batch(N, sizeof(Vt<T>), D);
    const size_t lds = sizeof(Vt<T>) * ((size_t)N * D * RP + tw_lds_entries(N, sizeof(Vt<T>)));
    dispatch((row_fast<T, FI, D>), dim3(total), dim3(kThreads), lds, s, args, woff, np);
}

template <typename T, int FI>
void launch_pencil_fast_d(int d, const PencilArgs *args, const int *woff, int np, int total, const Disp &s) {
    if (d == 3)
        launch_pencil_fast_t<T, FI, 3>(args, woff, np, total, s);
    else
        launch_pencil_fast_t<T, FI, 2>(args, woff, np, total, s);
}

template <typename T, int FI>
void launch_row_fast_d(int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    if (d == 3)
        launch_row_fast_t<T, FI, 3>(args, woff, np, total, s);
    else
        launch_row_fast_t<T, FI, 2>(args, woff, np, total, s);
}

template <typename T>
void launch_pencil_fast(int fi, int d, const PencilArgs *args, const int *woff, int np, int total,
                        const Disp &s) {
    switch (fi) {
        case 0: launch_pencil_fast_d<T, 0>(d, args, woff, np, total, s); break;
        case 1: launch_pencil_fast_d<T, 1>(d, args, woff, np, total, s); break;
        case 2: launch_pencil_fast_d<T, 2>(d, args, woff, np, total, s); break;
        case 3: launch_pencil_fast_d<T, 3>(d, args, woff, np, total, s); break;
        case 4: launch_pencil_fast_d<T, 4>(d, args, woff, np, total, s); break;
        default: launch_pencil_fast_d<T, 5>(d, args, woff, np, total, s); break;
    }
}

template <typename T>
void launch_row_fast(int fi, int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    switch (fi) {
        case 0: launch_row_fast_d<T, 0>(d, args, woff, np, total, s); break;
        case 1: launch_row_fast_d<T, 1>(d, args, woff, np, total, s); break;
        case 2: launch_row_fast_d<T, 2>(d, args, woff, np, total, s); break;
        case 3: launch_row_fast_d<T, 3>(d, args, woff, np, total, s); break;
        case 4: launch_row_fast_d<T, 4>(d, args, woff, np, total, s); break;
        default: launch_row_fast_d<T, 5>(d, args, woff, np, total, s); break;
    }
}


template <typename T, int FI>
void launch_row_iso_t(const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    if constexpr (palindromic(FI)) {
        constexpr int N = kFastSched[FI].n;
        if constexpr (kFastSched[FI].nst == 2) {
            const size_t lds = sizeof(T) * (size_t)split_tb(FI) * N + sizeof(Vt<T>) * N;
            dispatch((row_iso_split<T, FI>), dim3(total), dim3(split_nt(FI)), lds, s, args, woff, np);
        } else {
            const size_t lds = sizeof(Vt<T>) * ((size_t)iso_tb(FI) * N + tw_lds_entries(N, sizeof(Vt<T>)));
            dispatch((row_iso_fast<T, FI>), dim3(total), dim3(iso_nt(FI)), lds, s, args, woff, np);
        }
    }
}

template <typename T, int FI>
void launch_row_staged_t(int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    if constexpr (palindromic(FI) && kFastSched[FI].nst == 2) {
        if (d == 3)
            dispatch((row_iso_staged<T, FI, 3>), dim3(total), dim3(staged_nt(FI, 3, sizeof(Vt<T>))), staged_lds<T>(FI, 3),
                               s, args, woff, np);
        else
            dispatch((row_iso_staged<T, FI, 2>), dim3(total), dim3(staged_nt(FI, 2, sizeof(Vt<T>))), staged_lds<T>(FI, 2),
                               s, args, woff, np);
    }
}

template <typename T>
void launch_row_staged(int fi, int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    switch (fi) {
        case 0: launch_row_staged_t<T, 0>(d, args, woff, np, total, s); break;
        case 2: launch_row_staged_t<T, 2>(d, args, woff, np, total, s); break;
        default: break;
    }
}

template <typename T>
void launch_row_iso(int fi, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    switch (fi) {
        case 0: launch_row_iso_t<T, 0>(args, woff, np, total, s); break;
        case 1: launch_row_iso_t<T, 1>(args, woff, np, total, s); break;
        case 2: launch_row_iso_t<T, 2>(args, woff, np, total, s); break;
        case 3: launch_row_iso_t<T, 3>(args, woff, np, total, s); break;
        case 4: launch_row_iso_t<T, 4>(args, woff, np, total, s); break;
        default: launch_row_iso_t<T, 5>(args, woff, np, total, s); break;
    }
}


// Energy Gram quadrature (ROW_GRAM) for the specialised lengths: all d^2
// component fields of the d solutions are transformed to the grid in one
// in-place batch, then (A_M (E_s + e_s), E_t + e_t) is summed over the rows.
// Row pairs per work-group: one batch within 48 KB of LDS, so that several
// work-groups share a CU (a single pair of 225-point rows of 9 fields takes
// 32 KB in FP64: four work-groups per CU).
constexpr int gram_batch(int n, int es, int d) {
    int b = 8;
    while (b > 1 && d * d * b * n * es > 48 * 1024) b /= 2;
    return b;
}

template <typename T, int FI, int D>
__global__ __launch_bounds__(kThreads) void row_gram_fast(const RowArgs *__restrict__ ra, const int *__restrict__ woff,
                                                          int np) {
    using V = Vt<T>;
    constexpr int N = kFastSched[FI].n;
    constexpr int RP = gram_batch(N, sizeof(V), D);
    constexpr int NC = D * D;
    constexpr int NB = NC * RP;  // LDS layout [component][row pair][pos]
    int lb;
    const RowArgs &a = ra[find_problem(woff, np, &lb)];
    extern __shared__ __align__(16) unsigned char smem_raw[];  // 16-byte complex doubles
    V *X = reinterpret_cast<V *>(smem_raw);
    const int nh = a.Nh_row;
    const V *tw = reinterpret_cast<const V *>(a.tw) + a.f.twoff[0];
    const V *data = reinterpret_cast<const V *>(a.data);
    const T *g = reinterpret_cast<const T *>(a.g);
    const int pair0 = lb * RP;
    const int nvp = min(RP, (a.nrows + 1) / 2 - pair0);
    const V zero = mk<T>(T(0), T(0));
    // every global load of the work-group in flight at once: the half-spectrum
    // rows (at most (N + 1) / 2 points each) and, for the scalar-field form,
    // the material values of the accumulation below; the band of positions
    // no load writes is zeroed by a loop of its own
    constexpr int NHMAX = (N + 1) / 2;
    constexpr int PE = (NB * NHMAX + kThreads - 1) / kThreads;
    constexpr int GP = (RP * N + kThreads - 1) / kThreads;
    V u1v[PE], u2v[PE];
#pragma unroll
    for (int t = 0; t < PE; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        const int pc = idx / nh;
        const int kx = idx - pc * nh;
        const int c = pc / RP;
        const int j = pc - c * RP;
        const bool ok = idx < NB * nh && j < nvp;
        const int r1 = 2 * (pair0 + (ok ? j : 0));
        const bool two = ok && r1 + 1 < a.nrows;
        const long o1 = ok ? (long)c * a.cs + (long)r1 * nh + kx : 0L;
        const long o2 = two ? o1 + nh : 0L;  // in range even if the load is issued
        u1v[t] = ok ? data[o1] : zero;
        u2v[t] = two ? data[o2] : zero;
    }
    T gv1[GP], gv2[GP];
    const bool gpre = a.nfield == 1;
#pragma unroll
    for (int t = 0; t < GP; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        const int j = idx / N;
        const int x = idx - j * N;
        const bool ok = gpre && idx < RP * N && j < nvp;
        const bool two = ok && 2 * (pair0 + j) + 1 < a.nrows;
        const long r1 = 2 * (pair0 + (ok ? j : 0));
        const long i1 = ok ? r1 * N + x : 0L, i2 = two ? i1 + N : 0L;
        gv1[t] = ok ? g[i1] : T(0);
        gv2[t] = two ? g[i2] : T(0);
    }
    const int nzb = N - 2 * nh + 1;  // positions nh .. N - nh of every field
    for (int idx = threadIdx.x; idx < NB * nzb; idx += kThreads) {
        const int pc = idx / nzb;
        X[pc * N + nh + (idx - pc * nzb)] = zero;
    }
#pragma unroll
    for (int t = 0; t < PE; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        if (idx >= NB * nh) continue;
        const int pc = idx / nh;
        const int kx = idx - pc * nh;
        const V u1 = u1v[t], u2 = u2v[t];  // zero for idle row pairs
        if (kx == 0) {
            X[pc * N] = mk<T>(u1.x, u2.x);
        } else {
            X[pc * N + kx] = mk<T>(u1.x - u2.y, u1.y + u2.x);
            X[pc * N + N - kx] = mk<T>(u1.x + u2.y, u2.x - u1.y);
        }
    }
    __syncthreads();
    fft_ip<T, FI, 0, 1, 0, NB, true>(X, tw, T(1));
    T A0[D * D], Dm[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) {
        A0[i] = T(a.A0[i]);
        Dm[i] = T(a.D[i]);
    }
    double gs[D * D];
#pragma unroll
    for (int i = 0; i < D * D; ++i) gs[i] = 0.0;
#pragma unroll
    for (int t = 0; t < GP; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        if (idx >= RP * N) continue;
        const int j = idx / N;
        const int x = idx - j * N;
        if (j >= nvp) continue;
        const int r1 = 2 * (pair0 + j);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int r = r1 + half;
            if (r >= a.nrows) continue;
            T am[D * D];
            if (a.nfield > 1) {
                sym_load<T>(g, a.gstride, (long)r * N + x, D, am);
            } else {
                const T gg = half ? gv2[t] : gv1[t];
#pragma unroll
                for (int i = 0; i < D * D; ++i) am[i] = A0[i] + gg * Dm[i];
            }
            T f[D][D];
#pragma unroll
            for (int sol = 0; sol < D; ++sol)
#pragma unroll
                for (int b = 0; b < D; ++b) {
                    const V zv = X[((sol * D + b) * RP + j) * N + x];
                    f[sol][b] = (half ? zv.y : zv.x) + (sol == b ? T(1) : T(0));
                }
#pragma unroll
            for (int t = 0; t < D; ++t) {
                T af[D];
#pragma unroll
                for (int al = 0; al < D; ++al) {
                    T y = T(0);
#pragma unroll
                    for (int b = 0; b < D; ++b) y += am[al * D + b] * f[t][b];
                    af[al] = y;
                }
#pragma unroll
                for (int sol = 0; sol < D; ++sol) {
                    T dot = T(0);
#pragma unroll
                    for (int al = 0; al < D; ++al) dot += f[sol][al] * af[al];
                    gs[sol * D + t] += dot;
                }
            }
        }
    }
    block_sum_many<D * D>(gs, a.partial + (long)lb * D * D);
}

template <int FI, int D>
void launch_gram_fast_t(const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    constexpr int N = kFastSched[FI].n;
    constexpr int RP = gram_batch(N, 16, D);
    const size_t lds = (size_t)16 * N * D * D * RP;
    dispatch((row_gram_fast<double, FI, D>), dim3(total), dim3(kThreads), lds, s, args, woff, np);
}

template <int FI>
void launch_gram_fast_d(int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    if (d == 3)
        launch_gram_fast_t<FI, 3>(args, woff, np, total, s);
    else
        launch_gram_fast_t<FI, 2>(args, woff, np, total, s);
}

void launch_gram_fast(int fi, int d, const RowArgs *args, const int *woff, int np, int total, const Disp &s) {
    switch (fi) {
        case 0: launch_gram_fast_d<0>(d, args, woff, np, total, s); break;
        case 1: launch_gram_fast_d<1>(d, args, woff, np, total, s); break;
        case 2: launch_gram_fast_d<2>(d, args, woff, np, total, s); break;
        case 3: launch_gram_fast_d<3>(d, args, woff, np, total, s); break;
        case 4: launch_gram_fast_d<4>(d, args, woff, np, total, s); break;
        default: launch_gram_fast_d<5>(d, args, woff, np, total, s); break;
    }
}

// ---- multi-problem CG kernels (one problem per work-group for the scalar one) ----
__global__ __launch_bounds__(kThreads) void cg_check_multi_kernel(const CgItem *__restrict__ items) {
    const CgItem &it = items[blockIdx.x];
    CgStatus *st = it.st;
    if (!st->done) {
        const double rr = sum_fixed(it.rr_part, it.nrr);
        if (threadIdx.x == 0) {
            const int iter = st->iter + 1;
            st->iter = iter;
            if (it.hist != nullptr && iter < it.hist_cap) {
                it.hist[2 * iter] = rr;
                it.hist[2 * iter + 1] = st->alpha;
            }
            if (!isfinite(rr)) {
                st->breakdown = 1;
                st->done = 1;
            } else {
                // energy of the new iterate: one CG step lowers it by
                // alpha_k (r_{k-1}, r_{k-1})
                const double dstep = st->alpha * st->rr;
                st->energy -= dstep;
                st->beta = rr / st->rr;
                st->rr = rr;
                if (rr < st->rrmin) {
                    st->rrmin = rr;
                    st->rrmin_it = iter;
                }
                if (rr <= st->tol2 * st->rr0 || rr <= st->floor2) {
                    st->converged = 1;
                    st->done = 1;
                } else if (st->btol > 0.0 && iter >= 2 && st->dprev > 0.0 &&
                           dstep <= st->btol * fabs(st->energy) *
                                        (1.0 - fmin(fmax(dstep / st->dprev, 0.0), 0.99))) {
                    // bound test: the remaining decrease, estimated from the
                    // ratio q of the last two steps as dstep q / (1 - q), is
                    // below btol times the bound entry
                    st->converged = 1;
                    st->done = 1;
                } else if (iter >= st->maxit) {
                    st->done = 1;
                }
                st->dprev = dstep;
            }
        }
    }
    if (it.mirror != nullptr && threadIdx.x == 0) *it.mirror = *st;
}

// CG update: kUpdPer elements per thread in one pass (the grid, and with it
// the reduction order, depends only on the problem size).  Every work-group
// sums the (p, K p) partials of the projection pass itself, in one fixed
// order, while its vector loads are in flight, and forms alpha = (r, r) /
// (p, K p); work-group 0 records pq and alpha (or a breakdown) in the status.
constexpr int kUpdPer = 2;
template <typename T>
__global__ __launch_bounds__(kThreads) void cg_update_multi_kernel(const UpdArgs *__restrict__ ua,
                                                                   const int *__restrict__ woff, int np) {
    constexpr int U = kUpdPer;
    __shared__ double bcast;
    int lb;
    const UpdArgs &a = ua[find_problem(woff, np, &lb)];
    CgStatus *st = a.st;
    if (st->done) return;
    const double rr = st->rr;
    auto *x = gbl(reinterpret_cast<Vt<T> *>(a.x));
    auto *r = gbl(reinterpret_cast<Vt<T> *>(a.r));
    const auto *p = gbl(reinterpret_cast<const Vt<T> *>(a.p));
    const auto *q = gbl(reinterpret_cast<const Vt<T> *>(a.q));
    const int npc = (int)a.n_per_comp;
    const int total = npc * a.nc;
    // all loads of the thread's U elements in flight together
    T xx[U], xy[U], rx[U], ry[U], px[U], py[U], qx[U], qy[U];
    long off[U];
    int ii[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int idx = lb * (kThreads * U) + j * kThreads + threadIdx.x;
        const int c = idx / npc;
        ii[j] = idx - c * npc;
        off[j] = idx < total ? (long)c * a.cs + ii[j] : -1L;
        const long o = off[j] < 0 ? 0L : off[j];
        const Vt<T> xv = gld(x + o), rv = gld(r + o), pv = gld(p + o), qv = gld(q + o);
        xx[j] = xv.x;
        xy[j] = xv.y;
        rx[j] = rv.x;
        ry[j] = rv.y;
        px[j] = pv.x;
        py[j] = pv.y;
        qx[j] = qv.x;
        qy[j] = qv.y;
    }
    // the other shifts' contributions to K p, added in shift order
    for (int sh = 1; sh < a.nq; ++sh) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const long o = off[j] < 0 ? 0L : off[j];
            const Vt<T> qv = gld(q + sh * a.q_ss + o);
            qx[j] += qv.x;
            qy[j] += qv.y;
        }
    }
    const double pq = sum_fixed(a.pq_part, a.npq);
    if (threadIdx.x == 0) bcast = pq;
    __syncthreads();
    const double pqa = bcast;
    const bool bad = !(pqa > 0.0) || !isfinite(pqa);
    const double alpha_d = bad ? 0.0 : rr / pqa;
    if (lb == 0 && threadIdx.x == 0) {
        st->pq = pqa;
        if (bad) {
            // the material is SPD (validated when it is set), so with FP32
            // iterates a finite (p, K p) <= 0 after the first step is rounding
            // that has overtaken the iteration: a stall, and the best iterate
            // is kept; in FP64, or at the first step, the operator is at fault
            if (sizeof(T) == 4 && isfinite(pqa) && st->iter > 0)
                st->stagnated = 1;
            else
                st->breakdown = 1;
            st->done = 1;
        } else {
            st->alpha = alpha_d;
        }
    }
    if (bad) return;
    const T alpha = T(alpha_d);
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        if (off[j] < 0) continue;
        const T nxx = xx[j] + alpha * px[j], nxy = xy[j] + alpha * py[j];
        const T nrx = rx[j] - alpha * qx[j], nry = ry[j] - alpha * qy[j];
        gst(x + off[j], mk<T>(nxx, nxy));
        gst(r + off[j], mk<T>(nrx, nry));
        const double w = (ii[j] % a.Nh) == 0 ? 1.0 : 2.0;
        part += w * ((double)nrx * nrx + (double)nry * nry);
    }
    const double s = block_sum(part);
    if (threadIdx.x == 0) a.partial[lb] = s;
}

// ---------------------------------------------------------------------------
// Whole 2D CG solves, one work-group each (small double grids).  The CG
// vectors stay in registers (each thread owns coefficients idx = tid + 1024 j
// of the N0 x Nh half spectrum); the operator of Algorithm 2 runs on one
// complex M0 x M1 grid in LDS: the two components y_0, y_1 of the gradient
// field (real on the grid) are packed as z = y_0 + i y_1, so that
//   Z(k) = Y_0(k) + i Y_1(k),  Y_c(k) = i t_c(k) p(k)  (k_1 >= 0 stored;
//   Z(-k) = conj(Y_0(k)) + i conj(Y_1(k)) from the Hermitian symmetry),
// an inverse 2D DFT gives z on the grid, the material acts on (Re z, Im z) at
// every point, a forward 2D DFT gives Z', and
//   Y'_0(k) = (Z'(k) + conj(Z'(-k))) / 2,  Y'_1(k) = (Z'(k) - conj(Z'(-k))) / 2i
// feed the projection q(k) = -i scale sum_c t_c(k) Y'_c(k).  The CG update and
// the stopping test (as cg_update_multi_kernel and cg_check_multi_kernel,
// with work-group sums in a fixed order) follow in the same work-group, so a
// launch runs many iterations with no kernel boundary between them.
// ---------------------------------------------------------------------------
constexpr int kSoloNT = 1024;
template <typename T>
constexpr size_t solo_lds_bytes_t(int m0, int m1) {
    return sizeof(Vt<T>) * ((size_t)m0 * m1 + m0 + m1 + (m0 + 1) / 2);
}

// fixed-order sum over the 1024 threads (shuffle tree per wave, then the
// waves in turn by thread 0), broadcast to every thread
__device__ __forceinline__ double solo_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kSoloNT / 64; ++w) s += red[w];
        red[kSoloNT / 64] = s;
    }
    __syncthreads();
    return red[kSoloNT / 64];
}

template <typename T, int FI0, int FI1>
__global__ __launch_bounds__(kSoloNT) void solo2d_kernel(const SoloArgs *__restrict__ sa, int niter) {
    using V = Vt<T>;
    constexpr int M0 = kFastSched[FI0].n, M1 = kFastSched[FI1].n;
    constexpr int NT = kSoloNT;
    constexpr int CPT = ((M0 + 1) / 2 * ((M1 + 3) / 4) + NT - 1) / NT;  // coefficients per thread
    const SoloArgs &a = sa[blockIdx.x];
    __shared__ CgStatus S;
    __shared__ double red[NT / 64 + 1];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *Z = reinterpret_cast<V *>(smem_raw);  // [M0][M1]
    V *tw0 = Z + M0 * M1;                    // stage twiddles of axis 0
    V *tw1 = tw0 + M0;                       // and of axis 1
    V *P0 = tw1 + M1;                        // p at k_2 = 0, by stored index of k_1
    if (threadIdx.x == 0) S = *a.st;
    {
        const auto *t0 = gbl(reinterpret_cast<const V *>(a.tw) + a.tw0);
        const auto *t1 = gbl(reinterpret_cast<const V *>(a.tw) + a.tw1);
        for (int i = threadIdx.x; i < M0 - 1; i += NT) tw0[i] = gld(t0 + i);
        for (int i = threadIdx.x; i < M1 - 1; i += NT) tw1[i] = gld(t1 + i);
    }
    const int N0 = a.N0, Nh = a.Nh;
    const int ns = N0 * Nh;
    auto *gx = gbl(reinterpret_cast<V *>(a.x));
    auto *gr = gbl(reinterpret_cast<V *>(a.r));
    auto *gp = gbl(reinterpret_cast<V *>(a.p));
    T xr[CPT], xi[CPT], rr_[CPT], ri[CPT], pr[CPT], pi_[CPT], t0[CPT], t1[CPT], wgt[CPT];
    int zp[CPT], zm[CPT], lz[CPT];
    bool own[CPT], pos1[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int idx = threadIdx.x + j * NT;
        own[j] = idx < ns;
        const int id = own[j] ? idx : 0;
        const int l = id / Nh;
        const int k1 = id - l * Nh;
        const int k0 = wrapi(l, N0);
        T tb[2][3];
        const int nt = basis<T>(2, a.kind, k0, k1, 0, tb);
        t0[j] = nt ? tb[0][0] : T(0);
        t1[j] = nt ? tb[0][1] : T(0);
        pos1[j] = k1 > 0;
        lz[j] = k1 == 0 ? l : -1;
        wgt[j] = k1 == 0 ? T(1) : T(2);
        zp[j] = posmod(k0, M0) * M1 + k1;
        zm[j] = posmod(-k0, M0) * M1 + (k1 == 0 ? 0 : M1 - k1);
        const V vx = gld(gx + id), vr = gld(gr + id), vp = gld(gp + id);
        xr[j] = vx.x;
        xi[j] = vx.y;
        rr_[j] = vr.x;
        ri[j] = vr.y;
        pr[j] = vp.x;
        pi_[j] = vp.y;
    }
    const auto *g = gbl(reinterpret_cast<const T *>(a.g));
    const T A00 = T(a.A0[0]), A01 = T(a.A0[1]), A11 = T(a.A0[3]);
    const T D00 = T(a.D[0]), D01 = T(a.D[1]), D11 = T(a.D[3]);
    const T scale = T(a.scale);
    __syncthreads();
    for (int it = 0; it < niter && !S.done; ++it) {
        // p = r + beta p (beta = 0 at the first step of a solve)
        const T beta = T(S.beta);
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            pr[j] = rr_[j] + beta * pr[j];
            pi_[j] = ri[j] + beta * pi_[j];
            if (own[j] && lz[j] >= 0) P0[lz[j]] = mk<T>(pr[j], pi_[j]);
        }
        for (int i = threadIdx.x; i < M0 * M1; i += NT) Z[i] = mk<T>(T(0), T(0));
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (!own[j]) continue;
            // at k_2 = 0 the stored pair p(k_1, 0), p(-k_1, 0) enters through its
            // Hermitian part (p(k) + conj(p(-k))) / 2, the part a real field has
            // (as the per-pass kernels, whose real transform along the last
            // axis keeps the real part there); the rest, rounding of the
            // right-hand side, must not reach the field
            T px = pr[j], py = pi_[j];
            if (lz[j] >= 0) {
                const V pm = P0[lz[j] == 0 ? 0 : N0 - lz[j]];
                px = (px + pm.x) * T(0.5);
                py = (py - pm.y) * T(0.5);
            }
            // Y_c = i t_c p
            const T y0x = -t0[j] * py, y0y = t0[j] * px;
            const T y1x = -t1[j] * py, y1y = t1[j] * px;
            Z[zp[j]] = mk<T>(y0x - y1y, y0y + y1x);
            if (pos1[j]) Z[zm[j]] = mk<T>(y0x + y1y, y1x - y0y);
        }
        __syncthreads();
        // columns: only the N_2 = (M_2 + 1) / 2 non-zero ones (zero-padded
        // frequencies stay zero, and only they are read back after the
        // forward transform)
        fft_ip<T, FI0, 0, 1, 0, M1, false, NT, (M1 + 1) / 2>(Z, tw0, T(1));
        fft_ip<T, FI1, 0, 1, 0, M0, true, NT>(Z, tw1, T(1));
        if (a.nfield == 1) {
            for (int i = threadIdx.x; i < M0 * M1; i += NT) {
                const V z = Z[i];
                const T gv = g[i];
                const T a00 = A00 + gv * D00, a01 = A01 + gv * D01, a11 = A11 + gv * D11;
                Z[i] = mk<T>(a00 * z.x + a01 * z.y, a01 * z.x + a11 * z.y);
            }
        } else {
            for (int i = threadIdx.x; i < M0 * M1; i += NT) {
                const V z = Z[i];
                const T a00 = g[i], a01 = g[a.gstride + i], a11 = g[2 * a.gstride + i];
                Z[i] = mk<T>(a00 * z.x + a01 * z.y, a01 * z.x + a11 * z.y);
            }
        }
        __syncthreads();
        fft_ip<T, FI1, 0, 1, 0, M0, true, NT>(Z, tw1, T(-1));
        fft_ip<T, FI0, 0, 1, 0, M1, false, NT, (M1 + 1) / 2>(Z, tw0, T(-1));
        // projection q = -i scale sum_c t_c Y'_c and the partial of (p, q)
        T qr[CPT], qi[CPT];
        double part = 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            qr[j] = qi[j] = T(0);
            if (!own[j]) continue;
            const V zk = Z[zp[j]], zn = Z[zm[j]];
            const T h = T(0.5);
            const T y0x = (zk.x + zn.x) * h, y0y = (zk.y - zn.y) * h;
            const T y1x = (zk.y + zn.y) * h, y1y = (zn.x - zk.x) * h;
            const T s0 = t0[j] * scale, s1 = t1[j] * scale;
            qr[j] = s0 * y0y + s1 * y1y;
            qi[j] = -(s0 * y0x + s1 * y1x);
            part += (double)wgt[j] * ((double)pr[j] * (double)qr[j] + (double)pi_[j] * (double)qi[j]);
        }
        const double pq = solo_sum(part, red);
        const bool bad = !(pq > 0.0) || !isfinite(pq);
        if (threadIdx.x == 0) {
            S.pq = pq;
            if (bad) {
                // as the update pass: with FP32 iterates a finite (p, K p) <= 0
                // after the first step is a stall, otherwise a breakdown
                if (sizeof(T) == 4 && isfinite(pq) && S.iter > 0)
                    S.stagnated = 1;
                else
                    S.breakdown = 1;
                S.done = 1;
            } else {
                S.alpha = S.rr / pq;
            }
        }
        if (bad) break;  // uniform: pq is the same in every thread
        const double alpha_d = S.rr / pq;
        const T alpha = T(alpha_d);
        double part2 = 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (!own[j]) continue;
            xr[j] = xr[j] + alpha * pr[j];
            xi[j] = xi[j] + alpha * pi_[j];
            rr_[j] = rr_[j] - alpha * qr[j];
            ri[j] = ri[j] - alpha * qi[j];
            part2 += (double)wgt[j] * ((double)rr_[j] * rr_[j] + (double)ri[j] * ri[j]);
        }
        const double rr = solo_sum(part2, red);
        if (threadIdx.x == 0) {
            // the stopping test of cg_check_multi_kernel
            const int iter = S.iter + 1;
            S.iter = iter;
            if (a.hist != nullptr && iter < a.hist_cap) {
                a.hist[2 * iter] = rr;
                a.hist[2 * iter + 1] = S.alpha;
            }
            if (!isfinite(rr)) {
                S.breakdown = 1;
                S.done = 1;
            } else {
                const double dstep = S.alpha * S.rr;
                S.energy -= dstep;
                S.beta = rr / S.rr;
                S.rr = rr;
                if (rr < S.rrmin) {
                    S.rrmin = rr;
                    S.rrmin_it = iter;
                }
                if (rr <= S.tol2 * S.rr0 || rr <= S.floor2) {
                    S.converged = 1;
                    S.done = 1;
                } else if (S.btol > 0.0 && iter >= 2 && S.dprev > 0.0 &&
                           dstep <= S.btol * fabs(S.energy) * (1.0 - fmin(fmax(dstep / S.dprev, 0.0), 0.99))) {
                    S.converged = 1;
                    S.done = 1;
                } else if (iter >= S.maxit) {
                    S.done = 1;
                }
                S.dprev = dstep;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (!own[j]) continue;
        const int idx = threadIdx.x + j * NT;
        gst(gx + idx, mk<T>(xr[j], xi[j]));
        gst(gr + idx, mk<T>(rr_[j], ri[j]));
        gst(gp + idx, mk<T>(pr[j], pi_[j]));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *a.st = S;
        if (a.mirror != nullptr) *a.mirror = S;
    }
}

// ---- best-iterate checkpoints of the FP32-iteration form ----
// Every CG iterate is admissible, so its exact energy is a guaranteed bound
// (Sec. 6.4); with FP32 iterates the recursively updated residual and the
// iterate drift apart once rounding dominates, and the energy of later
// iterates rises again.  A checkpoint measures the exact energy of the
// current iterate x: with b = -G A_M E the right-hand side and K the operator,
// (A_M (E + x), E + x) = (A_M E, E) - 2 (b, x) + (K x, x).

// Partials of (b, x) over the update grid (half-spectrum weights).
template <typename T>
__global__ __launch_bounds__(kThreads) void ckpt_dot_kernel(UpdArgs a, const Vt<T> *b, double *part, int final) {
    const CgStatus *st = a.st;
    if (st->done && !final) return;
    const Vt<T> *x = reinterpret_cast<const Vt<T> *>(a.x);
    double acc = 0.0;
    const long total = a.n_per_comp * a.nc;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)a.nblocks * kThreads) {
        const long c = idx / a.n_per_comp;
        const long i = idx - c * a.n_per_comp;
        const long off = c * a.cs + i;
        const Vt<T> bv = b[off], xv = x[off];
        const double w = (i % a.Nh) == 0 ? 1.0 : 2.0;
        acc += w * ((double)bv.x * xv.x + (double)bv.y * xv.y);
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The energy of x against the best one; sets the copy / restore flags.
__global__ __launch_bounds__(kThreads) void ckpt_decide_kernel(CgStatus *st, const double *part_xkx, int n_xkx,
                                                               const double *part_bx, int n_bx, int window,
                                                               int final) {
    const bool skip = final ? (st->converged || st->breakdown) : st->done;
    if (skip) {
        if (threadIdx.x == 0) {
            st->ck_copy = 0;
            st->ck_restore = 0;
        }
        return;
    }
    const double xkx = sum_fixed(part_xkx, n_xkx);
    const double bx = sum_fixed(part_bx, n_bx);
    if (threadIdx.x != 0) return;
    const double e = st->eAE - 2.0 * bx + xkx;
    st->ck_copy = 0;
    st->ck_restore = 0;
    if (final) {
        // keep the current iterate unless the kept copy is better
        if (!(e <= st->ebest)) st->ck_restore = 1;
        return;
    }
    if (isfinite(e) && e < st->ebest) {
        st->ebest = e;
        st->best_it = st->iter;
        st->ck_copy = 1;
        return;
    }
    // a rise far beyond the rounding of the FP32 operator (~1e-7 of the
    // energy), or no gain while the residual has made no new minimum for a
    // whole window: the iteration has stalled
    const bool rise = !isfinite(e) || e > st->ebest + 1e-5 * fabs(st->ebest);
    const bool stall = st->iter - st->rrmin_it >= window;
    if (rise || stall) {
        st->stagnated = 1;
        st->done = 1;
        st->ck_restore = 1;
    }
}

// Copy x into xbest or back, as the checkpoint decided.
template <typename T>
__global__ __launch_bounds__(kThreads) void ckpt_copy_kernel(UpdArgs a, Vt<T> *xbest) {
    const CgStatus *st = a.st;
    const int cp = st->ck_copy, rs = st->ck_restore;
    if (!cp && !rs) return;
    Vt<T> *x = reinterpret_cast<Vt<T> *>(a.x);
    const long total = a.n_per_comp * a.nc;
    for (long idx = blockIdx.x * (long)kThreads + threadIdx.x; idx < total; idx += (long)a.nblocks * kThreads) {
        const long c = idx / a.n_per_comp;
        const long off = c * a.cs + (idx - c * a.n_per_comp);
        if (cp)
            xbest[off] = x[off];
        else
            x[off] = xbest[off];
    }
}

__global__ void copy_words_kernel(unsigned int *dst, const unsigned int *src, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ---- matrix voxel images (eq. gridcomp with C^p in R^{d x d}) ----
// Determinant and inverse of a symmetric 2 x 2 or 3 x 3 matrix by cofactors.
__device__ __forceinline__ double sym_det(const double *m, int d) {
    if (d == 2) return m[0] * m[3] - m[1] * m[2];
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

__device__ __forceinline__ void sym_inverse(const double *m, int d, double *out) {
    const double det = sym_det(m, d);
    if (d == 2) {
        out[0] = m[3] / det;
        out[1] = -m[1] / det;
        out[2] = -m[2] / det;
        out[3] = m[0] / det;
        return;
    }
    out[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    out[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    out[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    out[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    out[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    out[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    out[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    out[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    out[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

// A voxel matrix is accepted when finite, symmetric (to 1e-12 of its entries)
// and positive definite (leading principal minors > 0, Sylvester).
__global__ __launch_bounds__(kThreads) void tensor_check_kernel(const double *img, long n, int d, double *part) {
    double bad = 0.0;
    const int dd = d * d;
    for (long i = blockIdx.x * (long)kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
        double m[9];
        bool ok = true;
        for (int k = 0; k < dd; ++k) {
            m[k] = img[i * dd + k];
            ok = ok && isfinite(m[k]);
        }
        for (int r = 0; r < d && ok; ++r)
            for (int c = r + 1; c < d; ++c)
                if (fabs(m[r * d + c] - m[c * d + r]) > 1e-12 * (fabs(m[r * d + c]) + fabs(m[c * d + r]))) ok = false;
        if (ok) {
            const double m1 = m[0];
            const double m2 = m[0] * m[d + 1] - m[1] * m[d];
            ok = m1 > 0.0 && m2 > 0.0 && (d == 2 || sym_det(m, d) > 0.0);
        }
        bad += ok ? 0.0 : 1.0;
    }
    const double s = block_sum(bad);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kThreads) void tensor_component_kernel(const double *img, long n, int d, int a, int b,
                                                                    int invert, double *out) {
    const int dd = d * d;
    for (long i = blockIdx.x * (long)kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
        if (!invert) {
            out[i] = 0.5 * (img[i * dd + a * d + b] + img[i * dd + b * d + a]);
            continue;
        }
        double m[9], inv[9];
        for (int k = 0; k < dd; ++k) m[k] = img[i * dd + k];
        sym_inverse(m, d, inv);
        out[i] = 0.5 * (inv[a * d + b] + inv[b * d + a]);
    }
}

// Device-side validation of a voxel image: per work-group min, max and the
// number of entries that are not positive finite (part[3 b + 0..2]).
__global__ __launch_bounds__(kThreads) void image_stats_kernel(const double *img, long n, double *part) {
    double mn = INFINITY, mx = -INFINITY, bad = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = img[i];
        if (!(v > 0.0) || !isfinite(v)) {
            bad += 1.0;
        } else {
            mn = fmin(mn, v);
            mx = fmax(mx, v);
        }
    }
    __shared__ double smn[kThreads], smx[kThreads], sbd[kThreads];
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    sbd[threadIdx.x] = bad;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + w]);
            smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + w]);
            sbd[threadIdx.x] += sbd[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = smn[0];
        part[3 * blockIdx.x + 1] = smx[0];
        part[3 * blockIdx.x + 2] = sbd[0];
    }
}

// out[0..3] = min, max, #invalid, #entries equal to neither min nor max.
__global__ __launch_bounds__(kThreads) void image_stats_reduce(const double *part, int nb, double *out) {
    if (threadIdx.x == 0) {
        double mn = INFINITY, mx = -INFINITY, bad = 0.0;
        for (int b = 0; b < nb; ++b) {
            mn = fmin(mn, part[3 * b]);
            mx = fmax(mx, part[3 * b + 1]);
            bad += part[3 * b + 2];
        }
        out[0] = mn;
        out[1] = mx;
        out[2] = bad;
    }
}

__global__ __launch_bounds__(kThreads) void image_other_kernel(const double *img, long n, const double *mm,
                                                               double *part) {
    const double mn = mm[0], mx = mm[1];
    double cnt = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = img[i];
        if (v != mn && v != mx) cnt += 1.0;
    }
    const double s = block_sum(cnt);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
size_t pencil_lds_bytes(const PencilArgs &a, bool fp64) {
    const size_t es = fp64 ? 16 : 8;
    if (a.fast) return es * ((size_t)a.f.n * a.d * a.B + tw_lds_entries(a.f.n, (int)es));
    int lacc = 0;
    if (a.pro == PRO_EXPAND) lacc = a.nc * a.L_in;
    if (a.epi == EPI_PROJECT) lacc = a.nc * a.L_out;
    return es * ((size_t)2 * a.f.L * std::max(a.cb, 1) * a.B + (size_t)lacc * a.B + (size_t)std::max(a.twl, 0));
}

size_t row_lds_bytes(const RowArgs &a, bool fp64) {
    const size_t es = fp64 ? 16 : 8;
    if (a.fast == 3) {
        const int fi = fast_index(a.f.n);
        if (fi == 0) return fp64 ? staged_lds<double>(0, a.d) : staged_lds<float>(0, a.d);
        return fp64 ? staged_lds<double>(2, a.d) : staged_lds<float>(2, a.d);
    }
    if (a.fast == 2) {
        const int fi = fast_index(a.f.n);
        if (fi >= 0 && kFastSched[fi].nst == 2) return es / 2 * (size_t)a.RP * a.f.n + es * a.f.n;
        return es * ((size_t)a.RP * a.f.n + tw_lds_entries(a.f.n, (int)es));
    }
    if (a.fast)
        return es * ((size_t)a.f.n * (a.mode == ROW_GRAM ? a.d * a.d : a.d) * a.RP +
                     (a.mode == ROW_GRAM ? 0 : tw_lds_entries(a.f.n, (int)es)));
    const int nz = row_zbufs(a);
    return es * (size_t)(a.zbatch ? 2 * nz : nz + 1) * a.RP * a.f.L;
}

int pencil_grid_x(const PencilArgs &a) { return a.B > 0 ? (a.nb + a.B - 1) / a.B : 0; }
int row_grid(const RowArgs &a) {
    if (a.RP < 1) return 0;
    if (a.mode == ROW_GRAM && a.gpack && !a.fast) return (a.nrows + a.RP - 1) / a.RP;
    const int pairs = (a.nrows + 1) / 2;
    if (a.fast == 3) return (pairs + a.RP / a.d - 1) / (a.RP / a.d);
    return a.fast == 2 ? (a.d * pairs + a.RP - 1) / a.RP : (pairs + a.RP - 1) / a.RP;
}

static_assert(kNumFast == 6, "launch_*_fast switch covers six sizes");

void configure_pencil(PencilArgs &a, bool fp64) {
    const int fi = a.f.blue ? -1 : fast_index(a.f.n);
    bool ok = fi >= 0 && a.nsol == 1 && a.ncomp == a.d && a.epi != EPI_WINDOW && (a.d == 2 || a.d == 3) &&
              a.f.nst == kFastSched[fi].nst && a.L_in <= a.f.n && a.L_out <= a.f.n;
    for (int s = 0; ok && s < a.f.nst; ++s) ok = a.f.radix[s] == kFastSched[fi].r[s];
    if (ok) {
        a.fast = 1;
        a.B = pencil_batch(a.f.n, fp64 ? 16 : 8, a.d);
        return;
    }
    a.fast = 0;
    a.cb = 1;
    a.twl = 0;
    a.B = fp64 ? 8 : 16;
    while (a.B > 1 && pencil_lds_bytes(a, fp64) > kGenericLds) a.B /= 2;
    fit_pencil_components(a, fp64);
}

void fit_pencil_components(PencilArgs &a, bool fp64) {
    a.twl = 0;
    a.cb = std::max(a.ncomp, 1);
    while (a.cb > 1 && pencil_lds_bytes(a, fp64) > kGenericLds) --a.cb;
    // then the table in LDS, if it fits too: the stage twiddles (L - 1
    // entries), for Bluestein followed by the chirp (n) and the filter (L)
    if (a.f.nst < 1) return;
    a.twl = a.f.blue ? a.f.hoff + a.f.L - a.f.twoff[0] : a.f.L - 1;
    if (a.twl < 1 || pencil_lds_bytes(a, fp64) > kGenericLds) a.twl = 0;
}

void configure_row(RowArgs &r, bool fp64) {
    const int fi = r.f.blue ? -1 : fast_index(r.f.n);
    bool ok = fi >= 0 && (r.mode == ROW_OPER || r.mode == ROW_RHS) && r.ncomp == r.d && (r.d == 2 || r.d == 3) &&
              r.f.nst == kFastSched[fi].nst && r.Nh_row <= (r.f.n + 1) / 2;
    for (int s = 0; ok && s < r.f.nst; ++s) ok = r.f.radix[s] == kFastSched[fi].r[s];
    // the staged variant pays in FP64 (three waves per SIMD either way); in
    // FP32 its register count would cost occupancy
    if (ok && r.iso && r.mode == ROW_OPER && palindromic(fi) && kFastSched[fi].nst == 2 &&
        r.Nh_row <= staged_nhc(r.f.n)) {
        r.fast = 3;
        r.RP = staged_tb(fi == 0 ? 0 : 2, r.d, fp64 ? 16 : 8);
        return;
    }
    if (ok && r.iso && r.mode == ROW_OPER && palindromic(fi)) {
        r.fast = 2;
        r.RP = iso_tb(fi);
        return;
    }
    if (ok) {
        r.fast = 1;
        r.RP = fast_batch(r.f.n, fp64 ? 16 : 8, r.d);
        return;
    }
    const bool gram_ok = fi >= 0 && fp64 && r.mode == ROW_GRAM && r.ncomp == r.d * r.d && (r.d == 2 || r.d == 3) &&
                         r.f.nst == kFastSched[fi].nst && r.Nh_row <= (r.f.n + 1) / 2;
    bool sched = gram_ok;
    for (int s = 0; sched && s < r.f.nst; ++s) sched = r.f.radix[s] == kFastSched[fi].r[s];
    if (sched) {
        r.fast = 1;
        r.RP = gram_batch(r.f.n, 16, r.d);
        return;
    }
    r.fast = 0;
    r.zbatch = 0;
    r.gpack = 0;
    r.RP = 1;
    if (r.mode == ROW_GRAM && row_lds_bytes(r, fp64) > kGenericLds) r.gpack = 1;  // long rows: two components of one row per transform
    r.RP = 8;
    while (r.RP > 1 && row_lds_bytes(r, fp64) > kGenericLds) r.RP /= 2;
    fit_row_batch(r, fp64);
}

void fit_row_batch(RowArgs &r, bool fp64) {
    r.zbatch = 0;
    if (r.fast || r.gpack || row_zbufs(r) < 2) return;
    r.zbatch = 1;
    if (row_lds_bytes(r, fp64) > kGenericLds) r.zbatch = 0;
}

hipError_t launch_pencil(const PencilArgs &a, int nouter, bool fp64, hipStream_t s) {
    if (a.B < 1 || nouter < 1 || a.fast) return hipErrorInvalidValue;
    dim3 grid(pencil_grid_x(a), nouter);
    const size_t lds = pencil_lds_bytes(a, fp64);
    if (fp64) {
        hipLaunchKernelGGL(pencil_kernel<double>, grid, dim3(kThreads), lds, s, a);
    } else {
        hipLaunchKernelGGL(pencil_kernel<float>, grid, dim3(kThreads), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_row(const RowArgs &a, bool fp64, hipStream_t s) {
    if (a.RP < 1 || a.fast) return hipErrorInvalidValue;
    const size_t lds = row_lds_bytes(a, fp64);
    if (a.d != 2 && a.d != 3) return hipErrorInvalidValue;
    if (fp64) {
        if (a.d == 3)
            hipLaunchKernelGGL((row_kernel<double, 3>), dim3(row_grid(a)), dim3(kThreads), lds, s, a);
        else
            hipLaunchKernelGGL((row_kernel<double, 2>), dim3(row_grid(a)), dim3(kThreads), lds, s, a);
    } else {
        if (a.d == 3)
            hipLaunchKernelGGL((row_kernel<float, 3>), dim3(row_grid(a)), dim3(kThreads), lds, s, a);
        else
            hipLaunchKernelGGL((row_kernel<float, 2>), dim3(row_grid(a)), dim3(kThreads), lds, s, a);
    }
    return hipGetLastError();
}

bool solo_fits(int M0, int M1, bool fp64) {
    const int f0 = fast_index(M0), f1 = fast_index(M1);
    if (!((f0 == 0 || f0 == 1) && (f1 == 0 || f1 == 1))) return false;
    const size_t lds = fp64 ? solo_lds_bytes_t<double>(M0, M1) : solo_lds_bytes_t<float>(M0, M1);
    return lds + 1024 <= 160 * 1024;
}

template <typename T, int FI0, int FI1>
void launch_solo_t(const SoloArgs *args, int np, int niter, const Disp &s) {
    constexpr size_t lds = solo_lds_bytes_t<T>(kFastSched[FI0].n, kFastSched[FI1].n);
    if constexpr (lds + 1024 <= 160 * 1024)
        dispatch((solo2d_kernel<T, FI0, FI1>), dim3(np), dim3(kSoloNT), lds, s, args, niter);
}

template <typename T>
void launch_solo_d(int f0, int f1, const SoloArgs *args, int np, int niter, const Disp &s) {
    if (f0 == 0 && f1 == 0) launch_solo_t<T, 0, 0>(args, np, niter, s);
    if (f0 == 0 && f1 == 1) launch_solo_t<T, 0, 1>(args, np, niter, s);
    if (f0 == 1 && f1 == 0) launch_solo_t<T, 1, 0>(args, np, niter, s);
    if (f0 == 1 && f1 == 1) launch_solo_t<T, 1, 1>(args, np, niter, s);
}

hipError_t launch_solo(const SoloArgs &proto, const SoloArgs *args, int np, int niter, bool fp64, hipStream_t st,
                       LaunchEv ev) {
    if (np < 1 || niter < 1 || !solo_fits(proto.M0, proto.M1, fp64)) return hipErrorInvalidValue;
    const int f0 = fast_index(proto.M0), f1 = fast_index(proto.M1);
    const Disp s(st, ev);
    if (fp64)
        launch_solo_d<double>(f0, f1, args, np, niter, s);
    else
        launch_solo_d<float>(f0, f1, args, np, niter, s);
    return hipGetLastError();
}

int pencil_grid(const PencilArgs &a, int nouter) { return pencil_grid_x(a) * nouter; }
int update_blocks(long n) { return (int)std::max<long>(1, (n + (long)kThreads * kUpdPer - 1) / ((long)kThreads * kUpdPer)); }

hipError_t launch_pencil_multi(const PencilArgs &proto, const PencilArgs *args, const int *woff, int np, int total,
                               bool fp64, hipStream_t st, LaunchEv ev) {
    const int fi = fast_index(proto.f.n);
    if (!proto.fast || fi < 0 || np < 1 || total < 1) return hipErrorInvalidValue;
    const Disp s(st, ev);
    if (fp64)
        launch_pencil_fast<double>(fi, proto.d, args, woff, np, total, s);
    else
        launch_pencil_fast<float>(fi, proto.d, args, woff, np, total, s);
    return hipGetLastError();
}

hipError_t launch_row_multi(const RowArgs &proto, const RowArgs *args, const int *woff, int np, int total, bool fp64,
                            hipStream_t st, LaunchEv ev) {
    const int fi = fast_index(proto.f.n);
    if (!proto.fast || fi < 0 || np < 1 || total < 1) return hipErrorInvalidValue;
    const Disp s(st, ev);
    if (proto.mode == ROW_GRAM) {
        if (!fp64) return hipErrorInvalidValue;
        launch_gram_fast(fi, proto.d, args, woff, np, total, s);
        return hipGetLastError();
    }
    if (proto.fast == 3) {
        if (!(fi == 0 || fi == 2) || proto.mode != ROW_OPER) return hipErrorInvalidValue;
        if (fp64)
            launch_row_staged<double>(fi, proto.d, args, woff, np, total, s);
        else
            launch_row_staged<float>(fi, proto.d, args, woff, np, total, s);
        return hipGetLastError();
    }
    if (proto.fast == 2) {
        if (!palindromic(fi) || proto.mode != ROW_OPER) return hipErrorInvalidValue;
        if (fp64)
            launch_row_iso<double>(fi, args, woff, np, total, s);
        else
            launch_row_iso<float>(fi, args, woff, np, total, s);
        return hipGetLastError();
    }
    if (fp64)
        launch_row_fast<double>(fi, proto.d, args, woff, np, total, s);
    else
        launch_row_fast<float>(fi, proto.d, args, woff, np, total, s);
    return hipGetLastError();
}

hipError_t launch_cg_check_multi(const CgItem *items, int np, hipStream_t st, LaunchEv ev) {
    dispatch(cg_check_multi_kernel, dim3(np), dim3(kThreads), 0, Disp(st, ev), items);
    return hipGetLastError();
}

hipError_t launch_cg_update_multi(const UpdArgs *ua, const int *woff, int np, int total, bool fp64, hipStream_t st,
                                  LaunchEv ev) {
    const Disp s(st, ev);
    if (fp64)
        dispatch(cg_update_multi_kernel<double>, dim3(total), dim3(kThreads), 0, s, ua, woff, np);
    else
        dispatch(cg_update_multi_kernel<float>, dim3(total), dim3(kThreads), 0, s, ua, woff, np);
    return hipGetLastError();
}

hipError_t launch_cg_checkpoint(const UpdArgs &u, const void *b, void *xbest, const double *part_xkx, int n_xkx,
                                double *part_bx, int window, int final, bool fp64, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(ckpt_dot_kernel<double>, dim3(u.nblocks), dim3(kThreads), 0, s, u,
                           reinterpret_cast<const double2 *>(b), part_bx, final);
    else
        hipLaunchKernelGGL(ckpt_dot_kernel<float>, dim3(u.nblocks), dim3(kThreads), 0, s, u,
                           reinterpret_cast<const float2 *>(b), part_bx, final);
    hipLaunchKernelGGL(ckpt_decide_kernel, dim3(1), dim3(kThreads), 0, s, u.st, part_xkx, n_xkx, part_bx, u.nblocks,
                       window, final);
    if (fp64)
        hipLaunchKernelGGL(ckpt_copy_kernel<double>, dim3(u.nblocks), dim3(kThreads), 0, s, u,
                           reinterpret_cast<double2 *>(xbest));
    else
        hipLaunchKernelGGL(ckpt_copy_kernel<float>, dim3(u.nblocks), dim3(kThreads), 0, s, u,
                           reinterpret_cast<float2 *>(xbest));
    return hipGetLastError();
}

hipError_t launch_tensor_check(const double *img, long n, int d, double *part, int *nparts, hipStream_t s) {
    const int blocks = (int)std::max<long>(1, std::min<long>((n + kThreads - 1) / kThreads, 1024));
    *nparts = blocks;
    hipLaunchKernelGGL(tensor_check_kernel, dim3(blocks), dim3(kThreads), 0, s, img, n, d, part);
    return hipGetLastError();
}

hipError_t launch_tensor_component(const double *img, long n, int d, int a, int b, int invert, double *out,
                                   hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = (int)std::min<long>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(tensor_component_kernel, dim3(blocks), dim3(kThreads), 0, s, img, n, d, a, b, invert, out);
    return hipGetLastError();
}

hipError_t launch_copy_vec(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes % 4) return hipErrorInvalidValue;
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(copy_words_kernel, dim3(blocks), dim3(kThreads), 0, s, reinterpret_cast<unsigned int *>(dst),
                       reinterpret_cast<const unsigned int *>(src), n);
    return hipGetLastError();
}

hipError_t launch_cg_init(CgStatus *st, const double *rr_part, int n_rr, const double *load_part, int n_load,
                          const double *work_part, double inv_mtot, double tol, double floor_rel, int maxit,
                          double btol, double *hist, hipStream_t s) {
    hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(kThreads), 0, s, st, rr_part, n_rr, load_part, n_load, work_part,
                       inv_mtot, tol, floor_rel, maxit, btol, hist);
    return hipGetLastError();
}

hipError_t launch_warm_residual(const UpdArgs &u, double *part_rr, double *part_bx, double *part_rx, bool fp64,
                                hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(warm_residual_kernel<double>, dim3(u.nblocks), dim3(kThreads), 0, s, u, part_rr, part_bx,
                           part_rx);
    else
        hipLaunchKernelGGL(warm_residual_kernel<float>, dim3(u.nblocks), dim3(kThreads), 0, s, u, part_rr, part_bx,
                           part_rx);
    return hipGetLastError();
}

hipError_t launch_cg_init_warm(CgStatus *st, const double *part_rr, const double *part_bx, const double *part_rx,
                               int nparts, const double *scal, double mtot, double tol, double floor_rel, int maxit,
                               double btol, double *hist, hipStream_t s) {
    hipLaunchKernelGGL(cg_init_warm_kernel, dim3(1), dim3(kThreads), 0, s, st, part_rr, part_bx, part_rx, nparts,
                       scal, mtot, tol, floor_rel, maxit, btol, hist);
    return hipGetLastError();
}

hipError_t launch_sample_incl(double *g, int d, const int *M, const InclDev *inc, int n, double w0, hipStream_t s) {
    const int m0 = M[0], m1 = M[1], m2 = d == 3 ? M[2] : 1;
    const long total = (long)m0 * m1 * m2;
    const int blocks = (int)std::max<long>(1, std::min<long>(2048, (total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(sample_incl_kernel, dim3(blocks), dim3(kThreads), 0, s, g, d, m0, m1, m2, inc, n, w0);
    return hipGetLastError();
}

hipError_t launch_sample_voxel(double *g, const double *img, int d, const int *P, const int *M, int map, double vmax,
                               hipStream_t s) {
    const int m0 = M[0], m1 = M[1], m2 = d == 3 ? M[2] : 1;
    const int p0 = P[0], p1 = P[1], p2 = d == 3 ? P[2] : 1;
    const long total = (long)m0 * m1 * m2;
    const int blocks = (int)std::max<long>(1, std::min<long>(2048, (total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(sample_voxel_kernel, dim3(blocks), dim3(kThreads), 0, s, g, img, p0, p1, p2, m0, m1, m2, map,
                       vmax);
    return hipGetLastError();
}

hipError_t launch_envelope(double *upper, double *lower, int d, const int *P, const InclDev *inc, int n,
                           const double *ext, hipStream_t s) {
    const int p0 = P[0], p1 = P[1], p2 = d == 3 ? P[2] : 1;
    const long total = (long)p0 * p1 * p2;
    const int blocks = (int)std::max<long>(1, std::min<long>(2048, (total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(envelope_kernel, dim3(blocks), dim3(kThreads), 0, s, upper, lower, d, p0, p1, p2, inc, n, ext);
    return hipGetLastError();
}

hipError_t launch_fold_series(void *out, const void *coef, int d, const int *N, const int *L, int Lh,
                              const int *shift, hipStream_t s) {
    const int n0 = N[0], n1 = d == 3 ? N[1] : 1, n2 = N[d - 1];
    const long total = (d == 3 ? (long)n0 * n1 : (long)n0) * ((n2 + 1) / 2);
    const int blocks = (int)std::max<long>(1, std::min<long>(4096, (total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(fold_series_kernel, dim3(blocks), dim3(kThreads), 0, s, reinterpret_cast<double2 *>(out),
                       reinterpret_cast<const double2 *>(coef), d, n0, n1, n2, L[0], d == 3 ? L[1] : 1, Lh, shift[0],
                       d == 3 ? shift[1] : 0, shift[d - 1]);
    return hipGetLastError();
}

hipError_t launch_prolong(const void *src, bool src64, void *dst, bool dst64, int d, int nc, const int *Nf,
                          const int *Nc, hipStream_t s) {
    const int f1 = Nf[0], f2 = d == 3 ? Nf[1] : 1, f3h = (Nf[d - 1] + 1) / 2;
    const int c1 = Nc[0], c2 = d == 3 ? Nc[1] : 1, c3h = (Nc[d - 1] + 1) / 2;
    const long total = (long)f1 * f2 * f3h * nc;
    const int blocks = (int)std::max<long>(1, std::min<long>(1024, (total + kThreads - 1) / kThreads));
    if (src64 && dst64)
        hipLaunchKernelGGL((prolong_kernel<double, double>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const double2 *>(src), static_cast<double2 *>(dst), d, nc, f1, f2, f3h, c1, c2,
                           c3h);
    else if (src64)
        hipLaunchKernelGGL((prolong_kernel<double, float>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const double2 *>(src), static_cast<float2 *>(dst), d, nc, f1, f2, f3h, c1, c2,
                           c3h);
    else if (dst64)
        hipLaunchKernelGGL((prolong_kernel<float, double>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const float2 *>(src), static_cast<double2 *>(dst), d, nc, f1, f2, f3h, c1, c2,
                           c3h);
    else
        hipLaunchKernelGGL((prolong_kernel<float, float>), dim3(blocks), dim3(kThreads), 0, s,
                           static_cast<const float2 *>(src), static_cast<float2 *>(dst), d, nc, f1, f2, f3h, c1, c2,
                           c3h);
    return hipGetLastError();
}




hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    const size_t nw = bytes / 4;
    if (nw == 0) return hipSuccess;
    const int nb = (int)std::min<size_t>((nw + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nb), dim3(kThreads), 0, s, (unsigned int *)p, nw);
    return hipGetLastError();
}

hipError_t launch_convert_f2d(double *dst, const float *src, size_t n, hipStream_t s) {
    const int nb = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(f2d_kernel, dim3(nb), dim3(kThreads), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_convert_d2f(float *dst, const double *src, size_t n, hipStream_t s) {
    const int nb = (int)std::min<size_t>((n + kThreads - 1) / kThreads, 4096);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(d2f_kernel, dim3(nb), dim3(kThreads), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_sum_partials(double *out, const double *part, int nparts, int nvals, hipStream_t s) {
    if (nvals < 1) return hipSuccess;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(nvals), dim3(kThreads), 0, s, out, part, nparts, nvals);
    return hipGetLastError();
}

hipError_t launch_image_stats(const double *img, long n, double *part, double *out, hipStream_t s) {
    const int nb = 256;  // 3 * nb partials fit the plan's partial-sum region
    hipLaunchKernelGGL(image_stats_kernel, dim3(nb), dim3(kThreads), 0, s, img, n, part);
    hipLaunchKernelGGL(image_stats_reduce, dim3(1), dim3(kThreads), 0, s, part, nb, out);
    hipLaunchKernelGGL(image_other_kernel, dim3(nb), dim3(kThreads), 0, s, img, n, out, part);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kThreads), 0, s, out + 3, part, nb, 1);
    return hipGetLastError();
}

hipError_t launch_incl_coeff(void *out, int d, int L1, int L2, int Lh, const InclDev *incl, int n_incl,
                             double w0, hipStream_t s) {
    const long total = (d == 3 ? (long)L1 * L2 * Lh : (long)L1 * Lh);
    const int nb = (int)std::min<long>((total + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(incl_coeff_kernel, dim3(nb), dim3(kThreads), 0, s, (double2 *)out, d, L1, L2, Lh, incl,
                       n_incl, w0);
    return hipGetLastError();
}

}  // namespace fftgal
