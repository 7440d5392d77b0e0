// Mixed-radix (2, 3, 5) complex FFT building blocks for LDS-staged batched
// transforms along one grid axis.
//
// The pair densities of Eq. fft and the orbitals of Eq. get_wfs are 3-D DFTs on
// the real-space grid; every kernel here does them one axis at a time on lines
// held in LDS, as a sequence of self-sorting (Stockham) radix passes. A pass of
// radix R with Ns = product of the earlier radices reads element j + r N/R,
// multiplies by exp(dir 2 pi i r (j mod Ns)/(Ns R)), does an R-point DFT in
// registers and writes element (j - j mod Ns) R + j mod Ns + r Ns of the other
// buffer; after the last pass the line is in natural order.
//
// This header compiles as HIP device code and as plain host C++ (so the same
// arithmetic can be checked on a CPU).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RPA_HD __host__ __device__ __forceinline__
#else
#define RPA_HD inline
#endif

namespace rpa {

template <typename T>
struct cplx {
    T x, y;
};

template <typename T> RPA_HD cplx<T> mk(T x, T y) { cplx<T> r; r.x = x; r.y = y; return r; }
template <typename T> RPA_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T> RPA_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T> RPA_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> RPA_HD cplx<T> scale(cplx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T> RPA_HD cplx<T> conj(cplx<T> a) { return mk(a.x, -a.y); }
// conj(a) * b
template <typename T> RPA_HD cplx<T> cmulc(cplx<T> a, cplx<T> b) {
    return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// i * s * a  (s = +1 or -1)
template <int S, typename T> RPA_HD cplx<T> imul(cplx<T> a) { return S > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x); }

// ---------------------------------------------------------------------------
// products with constants known in double (roots of unity, 1/N). In FP32 a
// constant is held as two floats, hi = fl(c) and lo = fl(c - hi), and the
// product as x hi + x lo with one fused multiply-add: the result then carries
// only the rounding of the arithmetic, which differs from pair to pair and
// averages out in chi0, and not the representation error of the constant,
// which shifts every transform of every pair the same way (a bias of a few
// 1e-7 in |rho(G)|^2 with singly rounded constants). FP64 multiplies plainly.
// ---------------------------------------------------------------------------
template <typename T> struct Split2 {
    T hi, lo;
};
template <typename T> RPA_HD Split2<T> split2(double c) {
    Split2<T> r;
    r.hi = T(c);
    r.lo = sizeof(T) == 4 ? T(c - (double)r.hi) : T(0);
    return r;
}
template <typename T> RPA_HD T mulk(T x, Split2<T> c) {
    if constexpr (sizeof(T) == 4) return __builtin_fmaf(x, c.hi, x * c.lo);
    else return x * c.hi;
}
template <typename T> RPA_HD cplx<T> scalek(cplx<T> a, Split2<T> c) { return mk(mulk(a.x, c), mulk(a.y, c)); }
// a * (c + i s) with c, s split
template <typename T> RPA_HD cplx<T> cmulk(cplx<T> a, Split2<T> c, Split2<T> s) {
    if constexpr (sizeof(T) == 4) {
        const float rl = a.x * c.lo - a.y * s.lo, il = a.x * s.lo + a.y * c.lo;
        return mk(__builtin_fmaf(a.x, c.hi, __builtin_fmaf(-a.y, s.hi, rl)),
                  __builtin_fmaf(a.x, s.hi, __builtin_fmaf(a.y, c.hi, il)));
    } else {
        return a * mk(c.hi, s.hi);
    }
}
template <typename T> RPA_HD cplx<T> cmulk(cplx<T> a, double c, double s) {
    return cmulk(a, split2<T>(c), split2<T>(s));
}

// ---------------------------------------------------------------------------
// compile-time roots of unity: cos and sin of 2 pi e / R by Taylor series on
// the reduced argument (exact to double rounding for |x| <= pi).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ce_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double ce_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 40; ++n) {
        term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}

template <int R>
struct Roots {
    double c[R];
    double s[R];
    constexpr Roots() : c(), s() {
        for (int e = 0; e < R; ++e) {
            double ang = 2.0 * kPi * e / R;
            if (ang > kPi) ang -= 2.0 * kPi;
            c[e] = ce_cos(ang);
            s[e] = ce_sin(ang);
            // exact values on the axes keep symmetric terms symmetric
            if (e == 0) { c[e] = 1.0; s[e] = 0.0; }
            if (4 * e == R) { c[e] = 0.0; s[e] = 1.0; }
            if (2 * e == R) { c[e] = -1.0; s[e] = 0.0; }
            if (4 * e == 3 * R) { c[e] = 0.0; s[e] = -1.0; }
        }
    }
};

// ---------------------------------------------------------------------------
// small DFTs in registers: X_k = sum_n x_n exp(DIR 2 pi i n k / R)
// ---------------------------------------------------------------------------
template <int R, int DIR, typename T> struct Dft;

template <int DIR, typename T> struct Dft<2, DIR, T> {
    static RPA_HD void run(cplx<T>* v) {
        cplx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <int DIR, typename T> struct Dft<3, DIR, T> {
    static RPA_HD void run(cplx<T>* v) {
        const Split2<T> h = split2<T>(0.86602540378443864676372317075294);  // sin(2 pi/3)
        cplx<T> a = v[0], t1 = v[1] + v[2], t2 = v[1] - v[2];
        cplx<T> m = a - scale(t1, T(0.5));
        cplx<T> r = imul<DIR>(scalek(t2, h));
        v[0] = a + t1;
        v[1] = m + r;
        v[2] = m - r;
    }
};

template <int DIR, typename T> struct Dft<4, DIR, T> {
    static RPA_HD void run(cplx<T>* v) {
        cplx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
        cplx<T> s13 = v[1] + v[3], d13 = imul<DIR>(v[1] - v[3]);
        v[0] = s02 + s13;
        v[2] = s02 - s13;
        v[1] = d02 + d13;
        v[3] = d02 - d13;
    }
};

template <int DIR, typename T> struct Dft<5, DIR, T> {
    static RPA_HD void run(cplx<T>* v) {
        const Split2<T> c1 = split2<T>(0.30901699437494742410229341718282);   // cos(2 pi/5)
        const Split2<T> c2 = split2<T>(-0.80901699437494742410229341718282);  // cos(4 pi/5)
        const Split2<T> s1 = split2<T>(0.95105651629515357211643933337938);   // sin(2 pi/5)
        const Split2<T> s2 = split2<T>(0.58778525229247312916870595463907);   // sin(4 pi/5)
        cplx<T> a = v[0];
        cplx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
        cplx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
        cplx<T> m1 = a + scalek(t1, c1) + scalek(t2, c2);
        cplx<T> m2 = a + scalek(t1, c2) + scalek(t2, c1);
        cplx<T> r1 = imul<DIR>(scalek(t3, s1) + scalek(t4, s2));
        cplx<T> r2 = imul<DIR>(scalek(t3, s2) - scalek(t4, s1));
        v[0] = a + t1 + t2;
        v[1] = m1 + r1;
        v[4] = m1 - r1;
        v[2] = m2 + r2;
        v[3] = m2 - r2;
    }
};

// R = A*B by one Cooley-Tukey split: n = B n1 + n2, k = k1 + A k2.
template <int A, int B, int DIR, typename T>
RPA_HD void dft_split(cplx<T>* x) {
    constexpr int R = A * B;
    constexpr Roots<R> W{};
    cplx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        cplx<T> t[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
        Dft<A, DIR, T>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int e = (n2 * k1) % R;
            if (e == 0) {
                y[n2 * A + k1] = t[k1];
            } else {
                y[n2 * A + k1] = cmulk(t[k1], W.c[e], DIR * W.s[e]);
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cplx<T> t[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2 * A + k1];
        Dft<B, DIR, T>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = t[k2];
    }
}

template <int DIR, typename T> struct Dft<6, DIR, T> { static RPA_HD void run(cplx<T>* v) { dft_split<2, 3, DIR, T>(v); } };
template <int DIR, typename T> struct Dft<8, DIR, T> { static RPA_HD void run(cplx<T>* v) { dft_split<2, 4, DIR, T>(v); } };
template <int DIR, typename T> struct Dft<10, DIR, T> { static RPA_HD void run(cplx<T>* v) { dft_split<2, 5, DIR, T>(v); } };
template <int DIR, typename T> struct Dft<12, DIR, T> { static RPA_HD void run(cplx<T>* v) { dft_split<4, 3, DIR, T>(v); } };
template <int DIR, typename T> struct Dft<16, DIR, T> { static RPA_HD void run(cplx<T>* v) { dft_split<4, 4, DIR, T>(v); } };

// ---------------------------------------------------------------------------
// whole lines in registers: an N-point DFT (N = 2^a 3^b 5^c, known at compile
// time) by recursive Cooley-Tukey splits N = A * (N / A), A the first of 4, 3,
// 2, 5 dividing N. Every index and twiddle is a compile-time constant, so a
// thread holds its line in registers and no LDS or twiddle table is touched.
// ---------------------------------------------------------------------------
template <int N>
struct RegRadix {
    static constexpr int value = (N % 4 == 0 && N > 5) ? 4 : (N % 3 == 0) ? 3 : (N % 2 == 0) ? 2 : 5;
};

template <int N, int DIR, typename T> struct RegFft;

template <int A, int B, int DIR, typename T>
RPA_HD void reg_split(cplx<T>* x) {
    constexpr int R = A * B;
    constexpr Roots<R> W{};
    cplx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
        cplx<T> t[A];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
        Dft<A, DIR, T>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            const int e = (n2 * k1) % R;
            if (e == 0) {
                y[n2 * A + k1] = t[k1];
            } else {
                y[n2 * A + k1] = cmulk(t[k1], W.c[e], DIR * W.s[e]);
            }
        }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
        cplx<T> t[B];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2 * A + k1];
        RegFft<B, DIR, T>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = t[k2];
    }
}

template <int N, int DIR, typename T>
struct RegFft {
    static RPA_HD void run(cplx<T>* x) {
        if constexpr (N == 1) {
            (void)x;
        } else if constexpr (N == 2 || N == 3 || N == 4 || N == 5) {
            Dft<N, DIR, T>::run(x);
        } else {
            constexpr int A = RegRadix<N>::value;
            static_assert(N % A == 0, "register DFT length must be 2^a 3^b 5^c");
            reg_split<A, N / A, DIR, T>(x);
        }
    }
};

// Line lengths with register-resident kernels (other lengths use the LDS passes).
#define RPA_REG_SIZES(X) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64)

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
constexpr int kMaxStages = 8;

struct FftPlan {
    int n;
    int nstages;
    int radix[kMaxStages];
};

// Greedy factorisation into the supported radices, largest first. Returns
// false when n has a prime factor other than 2, 3, 5.
inline bool make_plan(int n, FftPlan* p) {
    static const int pref[] = {16, 12, 10, 8, 6, 5, 4, 3, 2};
    p->n = n;
    p->nstages = 0;
    if (n < 2) return false;
    int rem = n;
    while (rem > 1) {
        int pick = 0;
        for (int r : pref)
            if (rem % r == 0) { pick = r; break; }
        if (!pick || p->nstages == kMaxStages) return false;
        p->radix[p->nstages++] = pick;
        rem /= pick;
    }
    return true;
}

// entries of a twiddle table of an N-point axis: N, and N more low parts in FP32
template <typename T> RPA_HD int twiddle_len(int N) { return sizeof(T) == 4 ? 2 * N : N; }

// One Stockham pass over items [item0, item0 + nitems) with stride `step`.
// Work item w -> (line l, butterfly j); `line_fast` picks which index varies
// fastest across consecutive items. Element (l, e) lives at addr(l, e).
// `tw` holds exp(-2 pi i t / N) for t < N; in FP32 followed by the N low
// parts (twiddle_len entries in all).
template <int R, int DIR, typename T, class Addr>
RPA_HD void stockham_pass(const cplx<T>* in, cplx<T>* out, int N, int Ns, int nlines, bool line_fast,
                          Addr addr, const cplx<T>* tw, int item0, int step) {
    const int M = N / R;
    const int total = nlines * M;
    const int twstep = N / (Ns * R);
    for (int w = item0; w < total; w += step) {
        int l, j;
        if (line_fast) { l = w % nlines; j = w / nlines; }
        else { j = w % M; l = w / M; }
        const int k = j % Ns;
        cplx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = in[addr(l, j + r * M)];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int ti = r * k * twstep;
                cplx<T> t = tw[ti];
                if constexpr (sizeof(T) == 4) {
                    cplx<T> tl = tw[N + ti];
                    if (DIR > 0) {
                        t.y = -t.y;
                        tl.y = -tl.y;
                    }
                    v[r] = cmulk(v[r], Split2<T>{t.x, tl.x}, Split2<T>{t.y, tl.y});
                } else {
                    if (DIR > 0) t.y = -t.y;
                    v[r] = v[r] * t;
                }
            }
        }
        Dft<R, DIR, T>::run(v);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) out[addr(l, base + r * Ns)] = v[r];
    }
}

template <int DIR, typename T, class Addr>
RPA_HD void stockham_dispatch(int R, const cplx<T>* in, cplx<T>* out, int N, int Ns, int nlines,
                              bool line_fast, Addr addr, const cplx<T>* tw, int item0, int step) {
    switch (R) {
        case 2: stockham_pass<2, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 3: stockham_pass<3, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 4: stockham_pass<4, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 5: stockham_pass<5, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 6: stockham_pass<6, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 8: stockham_pass<8, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 10: stockham_pass<10, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 12: stockham_pass<12, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        case 16: stockham_pass<16, DIR>(in, out, N, Ns, nlines, line_fast, addr, tw, item0, step); break;
        default: break;
    }
}

}  // namespace rpa
