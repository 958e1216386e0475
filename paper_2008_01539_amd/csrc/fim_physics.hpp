// Cell properties with derivatives with respect to the cell's own
// unknowns (forward-mode dual numbers), for the three fluid families.
//
// Accumulation (Appendix A): M_c = PV(p) * (mass of component c per pore
// volume); PV(p) = pv_ref (1 + c_r (p - p_ref_rock)).  Phase flux
// coefficients (Appendix A, phase-potential upwinding): mob[c][l] is the
// mass of component c carried by phase l per unit potential drop and unit
// transmissibility, k_rl xi_{c,l} / mu_l; rho[l] is the phase mass density
// entering the gravity weight.
#pragma once

#include "fim_internal.hpp"

namespace fimk {

template <int N>
struct Dual {
    double v;
    double d[N];
};

template <int N>
__device__ inline Dual<N> dconst(double a) {
    Dual<N> r;
    r.v = a;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = 0.0;
    return r;
}

template <int N>
__device__ inline Dual<N> dvar(double a, int which) {
    Dual<N> r = dconst<N>(a);
    r.d[which] = 1.0;
    return r;
}

#define DUAL_BIN(OP, VEXPR, DEXPR)                                           \
    template <int N>                                                         \
    __device__ inline Dual<N> operator OP(const Dual<N>& a, const Dual<N>& b) { \
        Dual<N> r;                                                           \
        r.v = VEXPR;                                                         \
        _Pragma("unroll") for (int k = 0; k < N; k++) r.d[k] = DEXPR;        \
        return r;                                                            \
    }
DUAL_BIN(+, a.v + b.v, a.d[k] + b.d[k])
DUAL_BIN(-, a.v - b.v, a.d[k] - b.d[k])
DUAL_BIN(*, a.v * b.v, a.d[k] * b.v + a.v * b.d[k])
#undef DUAL_BIN

template <int N>
__device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r;
    const double inv = 1.0 / b.v;
    r.v = a.v / b.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
    return r;
}

template <int N>
__device__ inline Dual<N> operator*(double s, const Dual<N>& a) {
    Dual<N> r;
    r.v = s * a.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = s * a.d[k];
    return r;
}

template <int N>
__device__ inline Dual<N> operator+(double s, const Dual<N>& a) {
    Dual<N> r = a;
    r.v = s + a.v;
    return r;
}

template <int N>
__device__ inline Dual<N> operator-(double s, const Dual<N>& a) {
    Dual<N> r;
    r.v = s - a.v;
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = -a.d[k];
    return r;
}

template <int N>
__device__ inline Dual<N> operator-(const Dual<N>& a, double s) {
    Dual<N> r = a;
    r.v = a.v - s;
    return r;
}

template <int N>
__device__ inline Dual<N> dexp(const Dual<N>& a) {
    Dual<N> r;
    r.v = exp(a.v);
#pragma unroll
    for (int k = 0; k < N; k++) r.d[k] = r.v * a.d[k];
    return r;
}

// clamp to [0,1]: outside, a constant; on the interval (ends included), a
template <int N>
__device__ inline Dual<N> dclamp01(const Dual<N>& a) {
    if (a.v < 0.0) return dconst<N>(0.0);
    if (a.v > 1.0) return dconst<N>(1.0);
    return a;
}

template <int FK> struct FluidTraits;
template <> struct FluidTraits<1> { static constexpr int B = 1, NPH = 1; };
template <> struct FluidTraits<2> { static constexpr int B = 2, NPH = 2; };
template <> struct FluidTraits<3> { static constexpr int B = 3, NPH = 3; };

// which (component, phase) pairs carry mass
template <int FK>
__host__ __device__ constexpr bool carries(int c, int l) {
    return FK == 3 ? (c == l || (c == 2 && l == 1)) : (c == l);
}

template <int FK>
struct Props {
    static constexpr int B = FluidTraits<FK>::B, NPH = FluidTraits<FK>::NPH;
    Dual<B> M[B];
    Dual<B> rho[NPH];
    Dual<B> mob[B][NPH];
};

template <int FK>
__device__ inline void cell_props(const double* uu, int8_t status,
                                  double pv_ref, const DevFluid& f,
                                  Props<FK>& P) {
    constexpr int B = FluidTraits<FK>::B;
    using D = Dual<B>;
    const D p = dvar<B>(uu[0], 0);
    const D pv = pv_ref * (1.0 + f.c_r * (p - f.p_ref_rock));
    if constexpr (FK == 1) {
        const D rho = f.rho_ref * dexp(f.c * (p - f.p_ref));
        P.M[0] = pv * rho;
        P.rho[0] = rho;
        P.mob[0][0] = (1.0 / f.mu) * rho;
    } else if constexpr (FK == 2) {
        const D sw = dvar<B>(uu[1], 1);
        const D rw = f.rho_w * dexp(f.c_w * (p - f.p_ref));
        const D ro = f.rho_o * dexp(f.c_o * (p - f.p_ref));
        const D swn = dclamp01((1.0 / (1.0 - f.swc - f.sor)) * (sw - f.swc));
        const D krw = swn * swn;
        const D one_m = 1.0 - swn;
        const D kro = one_m * one_m;
        P.M[0] = pv * rw * sw;
        P.M[1] = pv * ro * (1.0 - sw);
        P.rho[0] = rw;
        P.rho[1] = ro;
        P.mob[0][0] = (1.0 / f.mu_w) * (rw * krw);
        P.mob[1][1] = (1.0 / f.mu_o) * (ro * kro);
        P.mob[0][1] = dconst<B>(0.0);
        P.mob[1][0] = dconst<B>(0.0);
    } else {
        const D sw = dvar<B>(uu[1], 1);
        const D x = dvar<B>(uu[2], 2);
        const bool sat = status == 1;
        const D rs_sat = (f.rs_b / f.p_b) * p;
        const D sg = sat ? x : dconst<B>(0.0);
        const D rs = sat ? rs_sat : x;
        const D so = (1.0 - sw) - sg;
        const D bo = (1.0 + f.bo_slope * rs) *
                     dexp(-f.c_o * (p - (f.p_b / f.rs_b) * rs));
        const D bg = dconst<B>(f.bg_c) / p;
        const D bw = dexp(-f.c_w * (p - f.p_ref));
        const D xw = dconst<B>(f.rho_wsc) / bw;
        const D xoo = dconst<B>(f.rho_osc) / bo;
        const D xgo = (f.rho_gsc * rs) / bo;
        const D xgg = dconst<B>(f.rho_gsc) / bg;
        const double is = 1.0 / f.span;
        const D aw = dclamp01(is * (sw - f.swc));
        const D ag = dclamp01(is * sg);
        const D ao = dclamp01(is * so);
        const D krw = aw * aw, krg = ag * ag, kro = ao * ao;
        P.M[0] = pv * sw * xw;
        P.M[1] = pv * so * xoo;
        P.M[2] = pv * (sg * xgg + so * xgo);
        P.rho[0] = xw;
        P.rho[1] = xoo + xgo;
        P.rho[2] = xgg;
        const D lw = (1.0 / f.mu_w) * krw, lo = (1.0 / f.mu_o) * kro,
                lg = (1.0 / f.mu_g) * krg;
#pragma unroll
        for (int c = 0; c < 3; c++)
#pragma unroll
            for (int l = 0; l < 3; l++) P.mob[c][l] = dconst<B>(0.0);
        P.mob[0][0] = xw * lw;
        P.mob[1][1] = xoo * lo;
        P.mob[2][1] = xgo * lo;
        P.mob[2][2] = xgg * lg;
    }
}

} // namespace fimk
