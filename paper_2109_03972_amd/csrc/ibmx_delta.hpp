// Regularized delta weights at the W stencil nodes of one marker axis.
//
// A marker at grid coordinate s = (X - origin)/h (nodes at i + 1/2) touches
// the nodes b .. b + W - 1.  With t the fractional offset defined below, the
// node distances are r_k = (b + k + 1/2) - s:
//   W = 3 (Sec. 2.1, eq. 3pt-stencil): b = floor(s) - 1, t = s - floor(s),
//          r_k = k - 1/2 - t.  All three phi_3(r_k) share the square root
//          q = sqrt(1 - 3 (1/2 - t)^2):
//          w0 = (7/2 - 3t - q)/6, w1 = (1 + q)/3, w2 = (1/2 + 3t - q)/6.
//   W = 4 (Sec. 2.2.3, eq. 4pt-stencil): b = floor(s - 1/2) - 1,
//          t = (s - 1/2) - floor(s - 1/2), r_k = k - 1 - t.  All four
//          phi_4(r_k) share q = sqrt(1 + 4t - 4t^2):
//          w0 = (3 - 2t - q)/8, w1 = (3 - 2t + q)/8,
//          w2 = (1 + 2t + q)/8, w3 = (1 + 2t - q)/8.
// The last node's weight vanishes exactly when t = 0.
// d/dX of a weight is (d/dt)/h since t grows with X at rate 1/h.
#pragma once

#include <hip/hip_runtime.h>

template <int W, typename T>
struct Delta;

template <typename T>
struct Delta<3, T> {
    static constexpr double base_shift = 0.0;   // b = floor(s - base_shift) - 1
    __device__ __forceinline__ static void w(T t, T *w)
    {
        const T d = T(0.5) - t;
        const T q = dev_sqrt<T>(T(1) - T(3) * d * d);
        w[0] = (T(3.5) - T(3) * t - q) * T(1.0 / 6.0);
        w[1] = (T(1) + q) * T(1.0 / 3.0);
        w[2] = (T(0.5) + T(3) * t - q) * T(1.0 / 6.0);
    }
    __device__ __forceinline__ static void wd(T t, T *w, T *dw)
    {
        const T d = T(0.5) - t;
        const T q = dev_sqrt<T>(T(1) - T(3) * d * d);
        const T dq = T(3) * d / q;
        w[0] = (T(3.5) - T(3) * t - q) * T(1.0 / 6.0);
        w[1] = (T(1) + q) * T(1.0 / 3.0);
        w[2] = (T(0.5) + T(3) * t - q) * T(1.0 / 6.0);
        dw[0] = (T(-3) - dq) * T(1.0 / 6.0);
        dw[1] = dq * T(1.0 / 3.0);
        dw[2] = (T(3) - dq) * T(1.0 / 6.0);
    }
};

template <typename T>
struct Delta<4, T> {
    static constexpr double base_shift = 0.5;
    __device__ __forceinline__ static void w(T t, T *w)
    {
        const T q = dev_sqrt<T>(T(1) + T(4) * t - T(4) * t * t);
        const T a = T(3) - T(2) * t, b = T(1) + T(2) * t;
        w[0] = (a - q) * T(0.125);
        w[1] = (a + q) * T(0.125);
        w[2] = (b + q) * T(0.125);
        w[3] = (b - q) * T(0.125);
    }
    __device__ __forceinline__ static void wd(T t, T *w, T *dw)
    {
        const T q = dev_sqrt<T>(T(1) + T(4) * t - T(4) * t * t);
        const T dq = (T(2) - T(4) * t) / q;
        const T a = T(3) - T(2) * t, b = T(1) + T(2) * t;
        w[0] = (a - q) * T(0.125);
        w[1] = (a + q) * T(0.125);
        w[2] = (b + q) * T(0.125);
        w[3] = (b - q) * T(0.125);
        dw[0] = (T(-2) - dq) * T(0.125);
        dw[1] = (T(-2) + dq) * T(0.125);
        dw[2] = (T(2) + dq) * T(0.125);
        dw[3] = (T(2) - dq) * T(0.125);
    }
};
