// device_common.h -- device-side building blocks shared by the HIP kernels:
// shape weights (Sec. II.D, Eqs. 17-18), Boris rotation (Sec. II.C,
// Eqs. 13-16), the Vay pusher and the Esirkepov stencil weights (Sec. II.E, Eqs. 20-22),
// templated on the real type so the FP32 and FP64 paths use one definition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// Component staggers in half cells: E_x, E_y, E_z, B_x, B_y, B_z (Yee cell,
// Sec. II.B).  sx/sy/sz[c] is 1 when component c sits half a cell up that axis.
__host__ __device__ constexpr int stag(int comp, int axis) {
    // rows: Ex Ey Ez Bx By Bz ; columns x y z
    return (comp == 0 && axis == 0) || (comp == 1 && axis == 1) || (comp == 2 && axis == 2) ||
                   (comp == 3 && axis != 0) || (comp == 4 && axis != 1) ||
                   (comp == 5 && axis != 2)
               ? 1
               : 0;
}

// Cell-integrated shape weights of order ORDER at position xi (cell units,
// stagger already subtracted): first node *i0 and ORDER+1 weights.
//   ORDER 1: integral of the unit top-hat -> (1-d, d) on floor(xi), floor(xi)+1
//   ORDER 2: integral of the triangle S_2 (Eq. 17) -> quadratic spline on the
//            nearest node and its two neighbours.
//   ORDER 4: integral of the cubic spline S_4 (Eq. 18) -> quartic spline on the
//            nearest node and two neighbours on each side.
template <int ORDER, typename R>
__device__ __forceinline__ void shape_weights(R xi, int &i0, R *w) {
    if constexpr (ORDER == 1) {
        R f = floor(xi);
        R d = xi - f;
        i0 = (int)f;
        w[0] = R(1) - d;
        w[1] = d;
    } else if constexpr (ORDER == 4) {
        // d in [-1/2, 1/2): ((1-2d)^4/384, (19-44d+24d^2+16d^3-16d^4)/96,
        // (115-120d^2+48d^4)/192, (19+44d+24d^2-16d^3-16d^4)/96, (1+2d)^4/384)
        R ic = floor(xi + R(0.5));
        R d = xi - ic;
        i0 = (int)ic - 2;
        const R d2 = d * d;
        const R m = R(1) - R(2) * d, p = R(1) + R(2) * d;
        const R m2 = m * m, p2 = p * p;
        w[0] = m2 * m2 * R(1.0 / 384.0);
        w[4] = p2 * p2 * R(1.0 / 384.0);
        const R even = R(19.0 / 96.0) + d2 * (R(0.25) - d2 * R(1.0 / 6.0));
        const R odd = d * (R(44.0 / 96.0) - d2 * R(1.0 / 6.0));
        w[1] = even - odd;
        w[3] = even + odd;
        w[2] = R(115.0 / 192.0) + d2 * (R(-0.625) + d2 * R(0.25));
    } else {
        // (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2); the last equals the
        // first plus d
        R ic = floor(xi + R(0.5));
        R d = xi - ic;
        i0 = (int)ic - 1;
        R a = R(0.5) - d;
        w[0] = (R(0.5) * a) * a;
        w[1] = R(0.75) - d * d;
        w[2] = w[0] + d;
    }
}

// 1/sqrt(x) and 1/x: the FP32 path uses the hardware approximations (v_rsq_f32,
// v_rcp_f32, about 1 ulp), the FP64 path the correctly rounded operations.
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }

// Boris push (Eqs. 13-16): u += q_m dt E/2; rotate about B with
// t = q_m dt B / (2 gamma(u^-)); u += q_m dt E/2.  `h` = q_m dt / 2.
template <typename R>
__device__ __forceinline__ void boris(R h, const R *E, const R *B, R *u) {
    R um0 = u[0] + h * E[0], um1 = u[1] + h * E[1], um2 = u[2] + h * E[2];
    R ig = rsqrt_r(R(1) + um0 * um0 + um1 * um1 + um2 * um2);
    R t0 = h * B[0] * ig, t1 = h * B[1] * ig, t2 = h * B[2] * ig;
    R f = R(2) * rcp_r(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
    R s0 = f * t0, s1 = f * t1, s2 = f * t2;
    R p0 = um0 + (um1 * t2 - um2 * t1);
    R p1 = um1 + (um2 * t0 - um0 * t2);
    R p2 = um2 + (um0 * t1 - um1 * t0);
    u[0] = um0 + (p1 * s2 - p2 * s1) + h * E[0];
    u[1] = um1 + (p2 * s0 - p0 * s2) + h * E[1];
    u[2] = um2 + (p0 * s1 - p1 * s0) + h * E[2];
}

// Vay pusher, the alternative Sec. II.C names for fields whose electric and
// magnetic forces nearly cancel (J.-L. Vay, Phys. Plasmas 15, 056701 (2008)):
// u^{n+1} - u^n = q_m dt (E + (v^n + v^{n+1})/2 x B) solved in closed form.
// With tau = h B (h = q_m dt / 2): u' = u + 2 h E + v x tau, u* = u'.tau,
// sigma = 1 + |u'|^2 - |tau|^2, gamma_new^2 the positive root of
// g^4 - sigma g^2 - (|tau|^2 + u*^2) = 0 (the form without cancellation for
// sigma < 0), t = tau / gamma_new, u = (u' + (u'.t) t + u' x t) / (1 + |t|^2).
template <typename R>
__device__ __forceinline__ void vay(R h, const R *E, const R *B, R *u) {
    const R ig0 = rsqrt_r(R(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const R v0 = u[0] * ig0, v1 = u[1] * ig0, v2 = u[2] * ig0;
    const R T0 = h * B[0], T1 = h * B[1], T2 = h * B[2];
    const R h2 = R(2) * h;
    const R p0 = u[0] + h2 * E[0] + (v1 * T2 - v2 * T1);
    const R p1 = u[1] + h2 * E[1] + (v2 * T0 - v0 * T2);
    const R p2 = u[2] + h2 * E[2] + (v0 * T1 - v1 * T0);
    const R tau2 = T0 * T0 + T1 * T1 + T2 * T2;
    const R us = p0 * T0 + p1 * T1 + p2 * T2;
    const R sigma = R(1) + p0 * p0 + p1 * p1 + p2 * p2 - tau2;
    const R k = tau2 + us * us;
    const R q = sqrt(sigma * sigma + R(4) * k);
    const R g2 = sigma >= R(0) ? R(0.5) * (sigma + q) : R(2) * k / (q - sigma);
    const R ig = rsqrt_r(g2);
    const R t0 = T0 * ig, t1 = T1 * ig, t2 = T2 * ig;
    const R sc = rcp_r(R(1) + t0 * t0 + t1 * t1 + t2 * t2);
    const R pt = p0 * t0 + p1 * t1 + p2 * t2;
    u[0] = sc * (p0 + pt * t0 + (p1 * t2 - p2 * t1));
    u[1] = sc * (p1 + pt * t1 + (p2 * t0 - p0 * t2));
    u[2] = sc * (p2 + pt * t2 + (p0 * t1 - p1 * t0));
}

// momentum update of the configured pusher (0 Boris, 1 Vay)
template <int PUSH, typename R>
__device__ __forceinline__ void push_u(R h, const R *E, const R *B, R *u) {
    if constexpr (PUSH == 1) vay<R>(h, E, B, u);
    else boris<R>(h, E, B, u);
}

// Esirkepov stencil along one axis: S0 (weights at the start of the move),
// DS = S1 - S0, on ORDER+2 nodes from *base = min of the two supports.
// xh, xe are start/end positions in cell units relative to any integer origin
// (integer nodes, no stagger); |xe - xh| < 1.
template <int ORDER, typename R>
__device__ __forceinline__ void esirkepov_axis(R xh, R xe, int &base, R *S0, R *DS) {
    constexpr int L = ORDER + 2;
    R wh[ORDER + 1], we[ORDER + 1];
    int ih, ie;
    shape_weights<ORDER>(xh, ih, wh);
    shape_weights<ORDER>(xe, ie, we);
    base = ih < ie ? ih : ie;
    const int oh = ih - base, oe = ie - base;  // 0 or 1
#pragma unroll
    for (int k = 0; k < L; ++k) {
        R a = R(0), b = R(0);
#pragma unroll
        for (int m = 0; m <= ORDER; ++m) {
            a = (k == m + oh) ? wh[m] : a;
            b = (k == m + oe) ? we[m] : b;
        }
        S0[k] = a;
        DS[k] = b - a;
    }
}

// Same stencil when the start-point weights wh (first node ih) are already
// known from the gather: only the end point is evaluated, and each node takes
// one select since the two supports are offset by 0 or 1 from `base`.
// `cross` is set when the two supports differ (ih != ie); otherwise node
// ORDER+1 of S0 and DS is zero and so is the running sum of DS at node ORDER.
template <int ORDER, typename R>
__device__ __forceinline__ void esirkepov_axis_from(int ih, const R *wh, R xe, int &base, R *S0,
                                                    R *DS, bool &cross) {
    constexpr int L = ORDER + 2;
    R we[ORDER + 1];
    int ie;
    shape_weights<ORDER>(xe, ie, we);
    base = ih < ie ? ih : ie;
    cross = ih != ie;
    const bool sh = ih > base, se = ie > base;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const R h0 = k <= ORDER ? wh[k] : R(0), h1 = k >= 1 ? wh[k - 1] : R(0);
        const R e0 = k <= ORDER ? we[k] : R(0), e1 = k >= 1 ? we[k - 1] : R(0);
        const R a = sh ? h1 : h0;
        S0[k] = a;
        DS[k] = (se ? e1 : e0) - a;
    }
}

__device__ __forceinline__ int wrap_index(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

}  // namespace pic
