// Local linear solve J_A x = -F_A (Section 4.3; the paper does not name a
// linear solver).  BiCGStab on the block-Jacobi scaled system
// A~ = D^{-1} J_A (D = diagonal blocks) inside FP64 iterative refinement:
//
//   r64 = -F - J x64            (FP64, unscaled)
//   solve A~ d = D^{-1} r64     (BiCGStab in precision T: float or double)
//   x64 += d                    until ||r64|| <= lin_rtol ||F||.
//
// One BiCGStab iteration is three fused kernels; each finishes its dot
// products with the last-block pattern and writes the scalars the next
// kernel needs into device memory, so no host round trip is needed inside
// an iteration.  Vector updates are fused into the matrix products: the
// product kernel rebuilds p (or s) for each neighbour from r, p, v on the
// fly, which saves a launch and a full vector pass.  Kernels return
// immediately once the solve is done, so the host can queue several
// iterations before it looks at the status.
#include "fim_device.hpp"

namespace fimk {

template <int B, typename T>
struct Vecs {
    T* x; T* r; T* rh; T* p_old; T* v_old; T* p_new; T* v_new; T* s; T* t;
};

// p_new = r + beta (p_old - omega v_old), rounded to T; used for the own
// row and for every neighbour so both see the same value
template <typename T>
__device__ inline double p_update(bool first, T r, T p, T v, double beta, double om) {
    const double x = first ? (double)r : (double)r + beta * ((double)p - om * (double)v);
    return (double)(T)x;
}
template <typename T>
__device__ inline double s_update(T r, T v, double al) {
    return (double)(T)((double)r - al * (double)v);
}

// --------------------------------------------- refinement residual + init
template <int B, typename T>
__global__ __launch_bounds__(NT) void k_ir_residual(int nA, LocalSys ls, KrylovBufs kb,
                                                    int x_zero, double lin_rtol,
                                                    double inner_rtol) {
    constexpr int BB = B * B;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    T* xT = (T*)kb.x;
    T* rr = (T*)kb.r;
    T* rh = (T*)kb.rh;
    double part[2] = {0.0, 0.0};
    if (r < nA) {
        double res[B];
#pragma unroll
        for (int c = 0; c < B; c++) res[c] = -ls.F[(long)r * B + c];
        if (!x_zero) {
            const int s = r / SLICE, lane = r % SLICE;
            const int base = ls.sptr[s];
            const int width = (ls.sptr[s + 1] - base) / SLICE;
            for (int k = 0; k < width; k++) {
                const long pos = (long)base + (long)k * SLICE + lane;
                const int cl = ls.col[pos];
                const double* a = ls.J + pos * BB;
#pragma unroll
                for (int c = 0; c < B; c++) {
                    double acc = 0.0;
#pragma unroll
                    for (int v = 0; v < B; v++) acc += a[c * B + v] * kb.x64[(long)cl * B + v];
                    res[c] -= acc;
                }
            }
        }
        const double* di = kb.dinv + (long)r * BB;
#pragma unroll
        for (int c = 0; c < B; c++) {
            kb.rir[(long)r * B + c] = res[c];
            part[0] += res[c] * res[c];
            double bt = 0.0;
#pragma unroll
            for (int v = 0; v < B; v++) bt += di[c * B + v] * res[v];
            const T btT = (T)bt;
            xT[(long)r * B + c] = (T)0;
            rr[(long)r * B + c] = btT;
            rh[(long)r * B + c] = btT;
            part[1] += (double)btT * (double)btT;
        }
    }
    block_sum<2>(part);
    if (threadIdx.x == 0) {
        kb.part[2 * blockIdx.x] = part[0];
        kb.part[2 * blockIdx.x + 1] = part[1];
    }
    if (last_block(&kb.sc->counter[0])) {
        double t[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
            t[0] += kb.part[2 * q];
            t[1] += kb.part[2 * q + 1];
        }
        block_sum<2>(t);
        if (threadIdx.x == 0) {
            KScal* sc = kb.sc;
            sc->rir2 = t[0];
            if (x_zero) {
                sc->fnorm2 = t[0];
                sc->target2 = lin_rtol * lin_rtol * t[0];
                sc->outer = 0;
            } else {
                sc->outer += 1;
            }
            const bool finite = isfinite(t[0]) && isfinite(t[1]);
            sc->outer_done = (!finite || t[0] <= sc->target2) ? 1 : 0;
            sc->breakdown = finite ? 0 : 1;
            sc->bnorm2 = t[1];
            sc->brk = sizeof(T) == 4 ? 1e-6 : 1e-14;
            sc->rho = t[1];
            sc->rho_prev = 1.0;
            sc->alpha = 1.0;
            sc->omega = 1.0;
            sc->iters = 0;
            double need = (t[0] > 0.0) ? 0.5 * sqrt(sc->target2 / t[0]) : 0.0;
            double inner = need > inner_rtol ? need : inner_rtol;
            sc->tol2 = inner * inner * t[1];
            sc->done = sc->outer_done;
            sc->counter[0] = 0;
        }
    }
}

// ----------------------------------------------- BiCGStab kernel A: v = A p
template <int B, typename T>
__global__ __launch_bounds__(NT) void k_bicg_a(int nA, LocalSys ls, const T* __restrict__ At,
                                               Vecs<B, T> V, KScal* __restrict__ sc,
                                               double* __restrict__ part) {
    if (sc->done) return;
    constexpr int BB = B * B;
    const bool first = sc->iters == 0;
    const double beta = first ? 0.0 : (sc->rho / sc->rho_prev) * (sc->alpha / sc->omega);
    const double om = sc->omega;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double dot[2] = {0.0, 0.0};
    if (r < nA) {
        double pi[B], vi[B];
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            pi[c] = p_update<T>(first, V.r[q], first ? V.r[q] : V.p_old[q],
                                first ? V.r[q] : V.v_old[q], beta, om);
            vi[c] = pi[c];
        }
        const int s = r / SLICE, lane = r % SLICE;
        const int base = ls.sptr[s];
        const int width = (ls.sptr[s + 1] - base) / SLICE;
        for (int k = 1; k < width; k++) {
            const long pos = (long)base + (long)k * SLICE + lane;
            const int cl = ls.col[pos];
            double pj[B];
#pragma unroll
            for (int c = 0; c < B; c++) {
                const long q = (long)cl * B + c;
                pj[c] = p_update<T>(first, V.r[q], first ? V.r[q] : V.p_old[q],
                                    first ? V.r[q] : V.v_old[q], beta, om);
            }
            const T* a = At + pos * BB;
#pragma unroll
            for (int c = 0; c < B; c++) {
                double acc = 0.0;
#pragma unroll
                for (int v = 0; v < B; v++) acc += (double)a[c * B + v] * pj[v];
                vi[c] += acc;
            }
        }
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            V.p_new[q] = (T)pi[c];
            const T vT = (T)vi[c];
            V.v_new[q] = vT;
            dot[0] += (double)V.rh[q] * (double)vT;
            dot[1] += (double)vT * (double)vT;
        }
    }
    block_sum<2>(dot);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dot[0];
        part[2 * blockIdx.x + 1] = dot[1];
    }
    if (last_block(&sc->counter[1])) {
        double t[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
            t[0] += part[2 * q];
            t[1] += part[2 * q + 1];
        }
        block_sum<2>(t);
        if (threadIdx.x == 0) {
            sc->sigma = t[0];
            // (r0, v) lost against |r0| |v|: the direction carries no
            // information in this precision; stop with the current x
            const double lim = sc->brk * sqrt(sc->bnorm2 * t[1]);
            const double al = sc->rho / t[0];
            if (!(fabs(t[0]) > lim) || !isfinite(al)) {
                sc->breakdown = 1;
                sc->done = 1;
            } else {
                sc->alpha = al;
            }
            sc->counter[1] = 0;
        }
    }
}

// ------------------------------------- kernel B: s = r - alpha v, t = A s
template <int B, typename T>
__global__ __launch_bounds__(NT) void k_bicg_b(int nA, LocalSys ls, const T* __restrict__ At,
                                               Vecs<B, T> V, KScal* __restrict__ sc,
                                               double* __restrict__ part) {
    if (sc->done) return;
    constexpr int BB = B * B;
    const double al = sc->alpha;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double dot[2] = {0.0, 0.0};
    if (r < nA) {
        double si[B], ti[B];
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            si[c] = s_update<T>(V.r[q], V.v_new[q], al);
            ti[c] = si[c];
        }
        const int s = r / SLICE, lane = r % SLICE;
        const int base = ls.sptr[s];
        const int width = (ls.sptr[s + 1] - base) / SLICE;
        for (int k = 1; k < width; k++) {
            const long pos = (long)base + (long)k * SLICE + lane;
            const int cl = ls.col[pos];
            double sj[B];
#pragma unroll
            for (int c = 0; c < B; c++) {
                const long q = (long)cl * B + c;
                sj[c] = s_update<T>(V.r[q], V.v_new[q], al);
            }
            const T* a = At + pos * BB;
#pragma unroll
            for (int c = 0; c < B; c++) {
                double acc = 0.0;
#pragma unroll
                for (int v = 0; v < B; v++) acc += (double)a[c * B + v] * sj[v];
                ti[c] += acc;
            }
        }
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            const T sT = (T)si[c], tT = (T)ti[c];
            V.s[q] = sT;
            V.t[q] = tT;
            dot[0] += (double)tT * (double)sT;
            dot[1] += (double)tT * (double)tT;
        }
    }
    block_sum<2>(dot);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dot[0];
        part[2 * blockIdx.x + 1] = dot[1];
    }
    if (last_block(&sc->counter[2])) {
        double t[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
            t[0] += part[2 * q];
            t[1] += part[2 * q + 1];
        }
        block_sum<2>(t);
        if (threadIdx.x == 0) {
            sc->ts = t[0];
            sc->tt = t[1];
            sc->omega = (t[1] > 0.0) ? t[0] / t[1] : 0.0;
            if (!isfinite(t[0]) || !isfinite(t[1])) {
                sc->breakdown = 1;
                sc->done = 1;
            }
            sc->counter[2] = 0;
        }
    }
}

// ----------------------- kernel C: x += alpha p + omega s, r = s - omega t
template <int B, typename T>
__global__ __launch_bounds__(NT) void k_bicg_c(int nA, Vecs<B, T> V, KScal* __restrict__ sc,
                                               double* __restrict__ part, int maxit) {
    if (sc->done) return;
    const double al = sc->alpha, om = sc->omega;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double dot[2] = {0.0, 0.0};
    if (r < nA) {
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            const double sv = (double)V.s[q];
            V.x[q] = (T)((double)V.x[q] + al * (double)V.p_new[q] + om * sv);
            const T rT = (T)(sv - om * (double)V.t[q]);
            V.r[q] = rT;
            dot[0] += (double)V.rh[q] * (double)rT;
            dot[1] += (double)rT * (double)rT;
        }
    }
    block_sum<2>(dot);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = dot[0];
        part[2 * blockIdx.x + 1] = dot[1];
    }
    if (last_block(&sc->counter[3])) {
        double t[2] = {0.0, 0.0};
        for (int q = threadIdx.x; q < (int)gridDim.x; q += blockDim.x) {
            t[0] += part[2 * q];
            t[1] += part[2 * q + 1];
        }
        block_sum<2>(t);
        if (threadIdx.x == 0) {
            sc->rho_prev = sc->rho;
            sc->rho = t[0];
            sc->rr = t[1];
            sc->iters += 1;
            if (t[1] <= sc->tol2 || sc->iters >= maxit) sc->done = 1;
            if (!isfinite(t[1]) || t[0] == 0.0 || sc->omega == 0.0) {
                sc->done = 1;
                if (t[1] > sc->tol2) sc->breakdown = 1;
            }
            sc->counter[3] = 0;
        }
    }
}

template <int B, typename T>
__global__ __launch_bounds__(NT) void k_ir_accumulate(int nA, double* __restrict__ x64,
                                                      const T* __restrict__ xT) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < (long)nA * B) x64[q] += (double)xT[q];
}

__global__ void k_copy_f64(double* __restrict__ d, const double* __restrict__ s, long n) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) d[q] = s[q];
}

void launch_copy_f64(double* dst, const double* src, long n, hipStream_t s) {
    if (n > 0) k_copy_f64<<<nblocks(n), NT, 0, s>>>(dst, src, n);
}

// ------------------------------------------------------------- launches
template <int B, typename T>
static Vecs<B, T> make_vecs(const KrylovBufs& kb, int parity) {
    Vecs<B, T> V;
    V.x = (T*)kb.x;
    V.r = (T*)kb.r;
    V.rh = (T*)kb.rh;
    V.p_old = (T*)kb.p[parity];
    V.v_old = (T*)kb.v[parity];
    V.p_new = (T*)kb.p[parity ^ 1];
    V.v_new = (T*)kb.v[parity ^ 1];
    V.s = (T*)kb.sv;
    V.t = (T*)kb.t;
    return V;
}

template <int B, typename T>
static void part_impl(int which, int nA, const LocalSys& ls, const KrylovBufs& kb,
                      int parity, int maxit, hipStream_t s) {
    const int nb = nblocks(nA);
    Vecs<B, T> V = make_vecs<B, T>(kb, parity);
    if (which == 0)
        k_bicg_a<B, T><<<nb, NT, 0, s>>>(nA, ls, (const T*)kb.At, V, kb.sc, kb.part);
    else if (which == 1)
        k_bicg_b<B, T><<<nb, NT, 0, s>>>(nA, ls, (const T*)kb.At, V, kb.sc, kb.part);
    else
        k_bicg_c<B, T><<<nb, NT, 0, s>>>(nA, V, kb.sc, kb.part, maxit);
}

void launch_ir_residual(int b, bool fp32, int nA, const LocalSys& ls,
                        const KrylovBufs& kb, bool x_zero, double lin_rtol,
                        double inner_rtol, hipStream_t s) {
    const int nb = nblocks(nA > 0 ? nA : 1);
#define IR(BV, TT) k_ir_residual<BV, TT><<<nb, NT, 0, s>>>(nA, ls, kb, x_zero ? 1 : 0, lin_rtol, inner_rtol)
    if (fp32) {
        if (b == 1) IR(1, float); else if (b == 2) IR(2, float); else IR(3, float);
    } else {
        if (b == 1) IR(1, double); else if (b == 2) IR(2, double); else IR(3, double);
    }
#undef IR
}

void launch_bicg_part(int which, int b, bool fp32, int nA, const LocalSys& ls,
                      const KrylovBufs& kb, int parity, int maxit, hipStream_t s) {
    if (nA <= 0) return;
    if (fp32) {
        if (b == 1) part_impl<1, float>(which, nA, ls, kb, parity, maxit, s);
        else if (b == 2) part_impl<2, float>(which, nA, ls, kb, parity, maxit, s);
        else part_impl<3, float>(which, nA, ls, kb, parity, maxit, s);
    } else {
        if (b == 1) part_impl<1, double>(which, nA, ls, kb, parity, maxit, s);
        else if (b == 2) part_impl<2, double>(which, nA, ls, kb, parity, maxit, s);
        else part_impl<3, double>(which, nA, ls, kb, parity, maxit, s);
    }
}

void launch_ir_accumulate(int b, bool fp32, int nA, const KrylovBufs& kb,
                          hipStream_t s) {
    if (nA <= 0) return;
    const int nb = nblocks((long)nA * b);
#define AC(BV, TT) k_ir_accumulate<BV, TT><<<nb, NT, 0, s>>>(nA, kb.x64, (const TT*)kb.x)
    if (fp32) {
        if (b == 1) AC(1, float); else if (b == 2) AC(2, float); else AC(3, float);
    } else {
        if (b == 1) AC(1, double); else if (b == 2) AC(2, double); else AC(3, double);
    }
#undef AC
}

} // namespace fimk
