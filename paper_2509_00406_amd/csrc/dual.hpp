// Second-order forward-mode active scalars for the element kernels (Sec. 5.1,
// Sec. 6.2: an active scalar carries its value and its derivatives with
// respect to a small, compile-time number K of local variables).
//
// Three scalar types share one set of overloaded operators so that every
// energy is written once and instantiated per evaluation mode (Sec. 6.2,
// last paragraph):
//   double         passive mode: value only
//   D1<K, T>       gradient-only mode: value + gradient
//   HD<K, T>       full mode: value + gradient + packed upper-triangle Hessian
//
// The primal value is always carried in FP64; the derivative channels use T
// (float or double). Small-strain shells put the primal quantities that the
// energies subtract (Green strain F^T F - I, dihedral angle minus its rest
// value) in a cancellation regime where an FP32 primal loses 3-4 digits;
// the derivative channels carry no such cancellation.
//
// All loops run over compile-time bounds and are fully unrolled: seeds are
// unit vectors known at compile time, so the compiler folds the zero entries
// of linear intermediates away.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace mad {

template <int K>
struct Packed {
    static constexpr int N = K * (K + 1) / 2;
    // index of (i, j), i <= j, in the row-major packed upper triangle
    __host__ __device__ static constexpr int at(int i, int j) {
        return i <= j ? i * K - (i * (i - 1)) / 2 + (j - i) : j * K - (j * (j - 1)) / 2 + (i - j);
    }
};

template <int K, typename T>
struct D1 {
    double v;
    T g[K];
};

template <int K, typename T>
struct HD {
    double v;
    T g[K];
    T h[Packed<K>::N];
};

// ---- construction ---------------------------------------------------------------------------
template <typename S> struct ScalarTraits;
template <> struct ScalarTraits<double> {
    static __device__ __forceinline__ double cst(double c) { return c; }
    static __device__ __forceinline__ double var(int, double v) { return v; }
};
template <int K, typename T> struct ScalarTraits<D1<K, T>> {
    static __device__ __forceinline__ D1<K, T> cst(double c) {
        D1<K, T> r;
        r.v = c;
#pragma unroll
        for (int i = 0; i < K; ++i) r.g[i] = T(0);
        return r;
    }
    static __device__ __forceinline__ D1<K, T> var(int idx, double v) {
        D1<K, T> r = cst(v);
#pragma unroll
        for (int i = 0; i < K; ++i) r.g[i] = (i == idx) ? T(1) : T(0);
        return r;
    }
};
template <int K, typename T> struct ScalarTraits<HD<K, T>> {
    static __device__ __forceinline__ HD<K, T> cst(double c) {
        HD<K, T> r;
        r.v = c;
#pragma unroll
        for (int i = 0; i < K; ++i) r.g[i] = T(0);
#pragma unroll
        for (int i = 0; i < Packed<K>::N; ++i) r.h[i] = T(0);
        return r;
    }
    static __device__ __forceinline__ HD<K, T> var(int idx, double v) {
        HD<K, T> r = cst(v);
#pragma unroll
        for (int i = 0; i < K; ++i) r.g[i] = (i == idx) ? T(1) : T(0);
        return r;
    }
};

template <typename S> __device__ __forceinline__ S cst(double c) { return ScalarTraits<S>::cst(c); }
template <typename S> __device__ __forceinline__ S var(int i, double v) { return ScalarTraits<S>::var(i, v); }

__device__ __forceinline__ double val(double a) { return a; }
template <int K, typename T> __device__ __forceinline__ double val(const D1<K, T>& a) { return a.v; }
template <int K, typename T> __device__ __forceinline__ double val(const HD<K, T>& a) { return a.v; }

// ---- D1 arithmetic ----------------------------------------------------------------------------
template <int K, typename T>
__device__ __forceinline__ D1<K, T> operator+(const D1<K, T>& a, const D1<K, T>& b) {
    D1<K, T> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = a.g[i] + b.g[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ D1<K, T> operator-(const D1<K, T>& a, const D1<K, T>& b) {
    D1<K, T> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = a.g[i] - b.g[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ D1<K, T> operator*(const D1<K, T>& a, const D1<K, T>& b) {
    D1<K, T> r;
    r.v = a.v * b.v;
    const T av = T(a.v), bv = T(b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = av * b.g[i] + bv * a.g[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ D1<K, T> operator*(const D1<K, T>& a, double c) {
    D1<K, T> r;
    r.v = a.v * c;
    const T cc = T(c);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = cc * a.g[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ D1<K, T> operator+(const D1<K, T>& a, double c) {
    D1<K, T> r = a;
    r.v = a.v + c;
    return r;
}
// f(a) with f0 = f(a.v), f1 = f'(a.v), f2 unused in first order
template <int K, typename T>
__device__ __forceinline__ D1<K, T> chain(const D1<K, T>& a, double f0, double f1, double) {
    D1<K, T> r;
    r.v = f0;
    const T d = T(f1);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = d * a.g[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ D1<K, T> chain2(const D1<K, T>& a, const D1<K, T>& b, double f0, double fa, double fb,
                                           double, double, double) {
    D1<K, T> r;
    r.v = f0;
    const T da = T(fa), db = T(fb);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = da * a.g[i] + db * b.g[i];
    return r;
}

// ---- HD arithmetic ----------------------------------------------------------------------------
template <int K, typename T>
__device__ __forceinline__ HD<K, T> operator+(const HD<K, T>& a, const HD<K, T>& b) {
    HD<K, T> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = a.g[i] + b.g[i];
#pragma unroll
    for (int i = 0; i < Packed<K>::N; ++i) r.h[i] = a.h[i] + b.h[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ HD<K, T> operator-(const HD<K, T>& a, const HD<K, T>& b) {
    HD<K, T> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = a.g[i] - b.g[i];
#pragma unroll
    for (int i = 0; i < Packed<K>::N; ++i) r.h[i] = a.h[i] - b.h[i];
    return r;
}
// product rule: (ab)'' = a b'' + b a'' + a' b'^T + b' a'^T
template <int K, typename T>
__device__ __forceinline__ HD<K, T> operator*(const HD<K, T>& a, const HD<K, T>& b) {
    HD<K, T> r;
    r.v = a.v * b.v;
    const T av = T(a.v), bv = T(b.v);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = av * b.g[i] + bv * a.g[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i; j < K; ++j) {
            const int p = Packed<K>::at(i, j);
            r.h[p] = av * b.h[p] + bv * a.h[p] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
        }
    return r;
}
template <int K, typename T>
__device__ __forceinline__ HD<K, T> operator*(const HD<K, T>& a, double c) {
    HD<K, T> r;
    r.v = a.v * c;
    const T cc = T(c);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = cc * a.g[i];
#pragma unroll
    for (int i = 0; i < Packed<K>::N; ++i) r.h[i] = cc * a.h[i];
    return r;
}
template <int K, typename T>
__device__ __forceinline__ HD<K, T> operator+(const HD<K, T>& a, double c) {
    HD<K, T> r = a;
    r.v = a.v + c;
    return r;
}
// unary chain rule: f(a)'' = f'(a) a'' + f''(a) a' a'^T
template <int K, typename T>
__device__ __forceinline__ HD<K, T> chain(const HD<K, T>& a, double f0, double f1, double f2) {
    HD<K, T> r;
    r.v = f0;
    const T d1 = T(f1), d2 = T(f2);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = d1 * a.g[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i; j < K; ++j) {
            const int p = Packed<K>::at(i, j);
            r.h[p] = d1 * a.h[p] + d2 * a.g[i] * a.g[j];
        }
    return r;
}
// binary chain rule for f(a, b) with partials fa, fb, faa, fbb, fab
template <int K, typename T>
__device__ __forceinline__ HD<K, T> chain2(const HD<K, T>& a, const HD<K, T>& b, double f0, double fa, double fb,
                                           double faa, double fbb, double fab) {
    HD<K, T> r;
    r.v = f0;
    const T da = T(fa), db = T(fb), daa = T(faa), dbb = T(fbb), dab = T(fab);
#pragma unroll
    for (int i = 0; i < K; ++i) r.g[i] = da * a.g[i] + db * b.g[i];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i; j < K; ++j) {
            const int p = Packed<K>::at(i, j);
            r.h[p] = da * a.h[p] + db * b.h[p] + daa * a.g[i] * a.g[j] + dbb * b.g[i] * b.g[j] +
                     dab * (a.g[i] * b.g[j] + b.g[i] * a.g[j]);
        }
    return r;
}

// ---- passive (double) counterparts ------------------------------------------------------------
__device__ __forceinline__ double chain(double, double f0, double, double) { return f0; }
__device__ __forceinline__ double chain2(double, double, double f0, double, double, double, double, double) {
    return f0;
}

// ---- elementary functions (primal and its derivatives in FP64) --------------------------------
template <typename S> __device__ __forceinline__ S sq(const S& a) { return a * a; }

template <typename S> __device__ __forceinline__ S dsqrt(const S& a) {
    const double v = val(a), s = sqrt(v);
    return chain(a, s, 0.5 / s, -0.25 / (s * v));
}

template <typename S> __device__ __forceinline__ S drecip(const S& a) {
    const double v = val(a), r = 1.0 / v;
    return chain(a, r, -r * r, 2.0 * r * r * r);
}

template <typename S> __device__ __forceinline__ S ddiv(const S& a, const S& b) { return a * drecip(b); }

// atan2(y, x) with its first and second partials
template <typename S> __device__ __forceinline__ S datan2(const S& y, const S& x) {
    const double yv = val(y), xv = val(x);
    const double r2 = xv * xv + yv * yv, ir2 = 1.0 / r2, ir4 = ir2 * ir2;
    return chain2(y, x, atan2(yv, xv), xv * ir2, -yv * ir2, -2.0 * xv * yv * ir4, 2.0 * xv * yv * ir4,
                  (yv * yv - xv * xv) * ir4);
}

}  // namespace mad
