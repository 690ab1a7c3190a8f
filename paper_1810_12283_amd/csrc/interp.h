// Interpolation weights of one grid axis (Sec. 3.1).
//
// A point at offset t in [0, 1] of its cell (left node c) takes the S stencil
// nodes c - H .. c + S - 1 - H, H = S / 2 - 1, with weights w_o(t) and their
// x-derivatives dw_o(t) = w_o'(t) / h, o = 0 .. S - 1:
//   S = 4: Keys' cubic convolution kernel with a = -1/2 (nodes c-1 .. c+2);
//   S = 6: the six-point quintic convolution kernel of Meijering et al. (1999),
//          the piecewise quintic on [-3, 3] that interpolates (1 at 0, 0 at the
//          other integers), is twice continuously differentiable and reproduces
//          polynomials up to degree four; these conditions fix it uniquely.
//          Node weights phi(t+2), phi(t+1), phi(t), phi(1-t), phi(2-t), phi(3-t)
//          with, on [0,1], [1,2], [2,3]:
//            1 - 5/4 x^2 - 35/12 x^3 + 21/4 x^4 - 25/12 x^5
//            -4 + 75/4 x - 245/8 x^2 + 545/24 x^3 - 63/8 x^4 + 25/24 x^5
//            18 - 153/4 x + 255/8 x^2 - 313/24 x^3 + 21/8 x^4 - 5/24 x^5
//          (the coefficient tables below are these polynomials expanded in t).
// Every weight is evaluated by Horner's rule with explicit fused multiply-adds
// (no contraction is left to the compiler), so the scatter, the gather, the
// pivoted Cholesky and the prediction kernels all get bitwise the same weights
// and the scatter stays the exact transpose of the gather.
#pragma once

#include <hip/hip_runtime.h>

namespace dski {

constexpr int kInterpCubic = 4;
constexpr int kInterpQuintic = 6;

template <int S>
struct InterpCoef;

// Keys cubic: w_o(t) = sum_k c[o][k] t^k
template <>
struct InterpCoef<4> {
  static constexpr int H = 1;
  static __device__ __forceinline__ double c(int o, int k) {
    constexpr double tab[4][4] = {
        {0.0, -0.5, 1.0, -0.5},
        {1.0, 0.0, -2.5, 1.5},
        {0.0, 0.5, 2.0, -1.5},
        {0.0, 0.0, -0.5, 0.5},
    };
    return tab[o][k];
  }
};

template <>
struct InterpCoef<6> {
  static constexpr int H = 2;
  static __device__ __forceinline__ double c(int o, int k) {
    constexpr double tab[6][6] = {
        {0.0, 1.0 / 12.0, -1.0 / 24.0, -3.0 / 8.0, 13.0 / 24.0, -5.0 / 24.0},
        {0.0, -2.0 / 3.0, 2.0 / 3.0, 13.0 / 8.0, -8.0 / 3.0, 25.0 / 24.0},
        {1.0, 0.0, -5.0 / 4.0, -35.0 / 12.0, 21.0 / 4.0, -25.0 / 12.0},
        {0.0, 2.0 / 3.0, 2.0 / 3.0, 11.0 / 4.0, -31.0 / 6.0, 25.0 / 12.0},
        {0.0, -1.0 / 12.0, -1.0 / 24.0, -11.0 / 8.0, 61.0 / 24.0, -25.0 / 24.0},
        {0.0, 0.0, 0.0, 7.0 / 24.0, -1.0 / 2.0, 5.0 / 24.0},
    };
    return tab[o][k];
  }
};

// Weights w[0..S) and x-derivatives dw[0..S) at offset t (ih = 1 / h).
template <int S>
__device__ __forceinline__ void interp_weights(double t, double ih, double* w, double* dw) {
  using C = InterpCoef<S>;
#pragma unroll
  for (int o = 0; o < S; ++o) {
    double v = C::c(o, S - 1);
    double d = (double)(S - 1) * C::c(o, S - 1);
#pragma unroll
    for (int k = S - 2; k >= 0; --k) {
      v = __builtin_fma(v, t, C::c(o, k));
      if (k >= 1) d = __builtin_fma(d, t, (double)k * C::c(o, k));
    }
    w[o] = v;
    dw[o] = d * ih;
  }
}

// Value weights only, or derivative weights only (deriv = true).
template <int S>
__device__ __forceinline__ void interp_weights_one(double t, double ih, bool deriv, double* w) {
  double v[S], d[S];
  interp_weights<S>(t, ih, v, d);
#pragma unroll
  for (int o = 0; o < S; ++o) w[o] = deriv ? d[o] : v[o];
}

}  // namespace dski
