// Local linear solve J_A x = -F_A (Section 4.3; the paper does not name a
// linear solver).  BiCGStab on the block-Jacobi scaled system
// A~ = D^{-1} J_A (D = diagonal blocks) inside FP64 iterative refinement:
//
//   r64 = -F - J x64            (FP64, unscaled)
//   solve A~ d = D^{-1} r64     (BiCGStab in precision T: float or double)
//   x64 += d                    until ||r64|| <= lin_rtol ||F||.
//
// One BiCGStab iteration is three kernels.  Each writes per-block partial
// dot products; the next kernel's blocks each reduce those partials in the
// same fixed order (so every block derives the same scalar, and the result
// is deterministic) before doing their rows.  No fences, atomics or extra
// finishing launches are needed: kernel boundaries order everything.  Block
// 0 also records the scalars (rho, alpha, omega, done, iters) for later
// kernels and for the host, which looks at them once per block of queued
// iterations.  Vector updates are fused into the matrix products: the
// product kernel rebuilds p (or s) for each neighbour from r, p, v on the
// fly, saving a launch and a vector pass.  Grids are capped at KB_MAXB
// blocks of KB_NT threads (grid-stride over rows) so that a partial array
// has at most KB_MAXB entries.
#include <hip/hip_ext.h>

#include "fim_device.hpp"

namespace fimk {

template <int B, typename T>
struct Vecs {
    T* x; T* r; T* rh; T* p_old; T* v_old; T* p_new; T* v_new; T* s; T* t;
};

template <int B, typename T>
__host__ __device__ inline Vecs<B, T> make_vecs(const KrylovBufs& kb, int parity) {
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

// Raw operands of one row of a product kernel: the slice geometry, the
// column indices and blocks of the first UNR off-diagonal slots and the
// values of NV source vectors at the row itself and at those neighbours.
// They are fetched before the iteration's scalars are known, so the
// fetches overlap the reduction of the previous kernel's partial sums; a
// row then waits for about two memory round trips (columns, then gathers
// and blocks) instead of two per slot.
constexpr int UNR = 8;
template <int B, typename T, int NV>
struct RowRaw {
    int base, width, lane;
    int cl[UNR];
    T a[UNR][B * B];
    T xn[NV][UNR][B];
    T xo[NV][B];
};

template <int B, typename T, int NV>
__device__ inline void fetch_row(const LocalSys& ls, const T* __restrict__ At, int r,
                                 const T* const* src, RowRaw<B, T, NV>& R) {
    constexpr int BB = B * B;
    const int s = r / SLICE;
    R.lane = r % SLICE;
    R.base = ls.sptr[s];
    R.width = (ls.sptr[s + 1] - R.base) / SLICE;
#pragma unroll
    for (int v = 0; v < NV; v++)
#pragma unroll
        for (int c = 0; c < B; c++) R.xo[v][c] = src[v][(long)r * B + c];
#pragma unroll
    for (int u = 0; u < UNR; u++) {
        const int k = 1 + u;   // k < width is uniform over the wave (one slice)
        R.cl[u] = (k < R.width) ? ls.col[(long)R.base + (long)k * SLICE + R.lane] : r;
    }
#pragma unroll
    for (int u = 0; u < UNR; u++) {
        const int k = 1 + u;
        if (k < R.width) {
            const T* ap = At + ((long)R.base + (long)k * SLICE + R.lane) * BB;
#pragma unroll
            for (int q = 0; q < BB; q++) R.a[u][q] = ap[q];
#pragma unroll
            for (int v = 0; v < NV; v++)
#pragma unroll
                for (int c = 0; c < B; c++) R.xn[v][u][c] = src[v][(long)R.cl[u] * B + c];
        } else {
#pragma unroll
            for (int q = 0; q < BB; q++) R.a[u][q] = (T)0;
#pragma unroll
            for (int v = 0; v < NV; v++)
#pragma unroll
                for (int c = 0; c < B; c++) R.xn[v][u][c] = (T)0;
        }
    }
}

// y += sum_k A~_rk x_k with x_k = f(raw source values at neighbour k);
// slots past the first UNR (wide rows) are loaded here directly
template <int B, typename T, int NV, class FX>
__device__ inline void finish_row(const LocalSys& ls, const T* __restrict__ At,
                                  const T* const* src, const RowRaw<B, T, NV>& R,
                                  double (&y)[B], FX fx) {
    constexpr int BB = B * B;
#pragma unroll
    for (int u = 0; u < UNR; u++) {
        if (1 + u >= R.width) break;
        T raw[NV][B];
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int c = 0; c < B; c++) raw[v][c] = R.xn[v][u][c];
        double xj[B];
        fx(raw, xj);
#pragma unroll
        for (int c = 0; c < B; c++) {
            double acc = 0.0;
#pragma unroll
            for (int v = 0; v < B; v++) acc += (double)R.a[u][c * B + v] * xj[v];
            y[c] += acc;
        }
    }
    for (int k = 1 + UNR; k < R.width; k++) {
        const long pos = (long)R.base + (long)k * SLICE + R.lane;
        const int cl = ls.col[pos];
        T raw[NV][B];
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int c = 0; c < B; c++) raw[v][c] = src[v][(long)cl * B + c];
        double xj[B];
        fx(raw, xj);
        const T* ap = At + pos * BB;
#pragma unroll
        for (int c = 0; c < B; c++) {
            double acc = 0.0;
#pragma unroll
            for (int v = 0; v < B; v++) acc += (double)ap[c * B + v] * xj[v];
            y[c] += acc;
        }
    }
}

static inline int kgrid(long rows) {
    long g = (rows + KB_NT - 1) / KB_NT;
    if (g < 1) g = 1;
    return (int)(g < KB_MAXB ? g : KB_MAXB);
}

// --------------------------------------------- refinement residual + init
// r64 = -F - J x64 (x64 skipped when zero), b~ = D^{-1} r64; x = 0,
// r = rh = b~.  Partials: ir[q] = (|r64|^2, |b~|^2); pc[q] = ((rh,r), (r,r))
// so that the first BiCGStab kernel finds rho_0 where it looks for rho.
template <int B, typename T>
__global__ __launch_bounds__(KB_NT) void k_ir_residual(const KSeg* __restrict__ segs,
                                                       const int* __restrict__ blk_seg,
                                                       int x_zero) {
    const KSeg& S = segs[blk_seg[blockIdx.x]];
    if (!S.active) return;
    const int lb = blockIdx.x - S.blk0, nbk = S.nblk, nA = S.nA;
    const LocalSys& ls = S.ls;
    const KrylovBufs& kb = S.kb;
    constexpr int BB = B * B;
    T* xT = (T*)kb.x;
    T* rr = (T*)kb.r;
    T* rh = (T*)kb.rh;
    double part[2] = {0.0, 0.0};
    for (int r = lb * blockDim.x + threadIdx.x; r < nA; r += nbk * blockDim.x) {
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
        kb.part_ir[2 * lb] = part[0];
        kb.part_ir[2 * lb + 1] = part[1];
        kb.part_c[4 * lb] = part[1];      // (rh, r_0) = |b~|^2
        kb.part_c[4 * lb + 1] = part[1];
        kb.part_c[4 * lb + 2] = 0.0;
        kb.part_c[4 * lb + 3] = 0.0;
    }
    if (lb == 0 && threadIdx.x == 0) {
        kb.sc->done = 0;
        kb.sc->iters = 0;
        kb.sc->breakdown = 0;
    }
}

// ------------------------------------------------------ kernel P (iter i)
// Finishes iteration i-1 and starts iteration i:
//   omega = (t,s)/(t,t), rho_i = (rh,s) - omega (rh,t)   [from kernel S]
//   x += alpha p + omega s;  r_i = s - omega t           [own rows]
//   p_i = r_i + beta (p_{i-1} - omega v_{i-1});  v_i = A~ p_i
// with p_i at the neighbours rebuilt from s, t, p, v on the fly.  Partial
// sums: (rh, v_i), (v_i, v_i), (r_i, r_i).  At i = 0, p_0 = r_0 (the
// refinement initialisation).  Stops (after the x, r update) at the
// iteration cap or when omega = 0.
template <int B, typename T, bool FIRST>
__global__ __launch_bounds__(KB_NT) void k_bicg_p(const KSeg* __restrict__ segs,
                                                  const int* __restrict__ blk_seg, int it) {
    const KSeg& S = segs[blk_seg[blockIdx.x]];
    if (!S.active) return;
    const int lb = blockIdx.x - S.blk0, nbk = S.nblk, nA = S.nA;
    const LocalSys& ls = S.ls;
    const T* __restrict__ At = (const T*)S.kb.At;
    const Vecs<B, T> V = make_vecs<B, T>(S.kb, it & 1);
    KScal* __restrict__ sc = S.kb.sc;
    const double* __restrict__ pin = FIRST ? S.kb.part_c : S.kb.part_b;
    double* __restrict__ pa = S.kb.part_a;
    const int done = sc->done;
    const double rho_prev = FIRST ? 1.0 : sc->rho_hist[(it - 1) & 1];
    const double al_prev = sc->alpha;
    constexpr int NR = FIRST ? 1 : 4;
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nbk; q += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; k++) red[k] += pin[(long)q * 4 + k];
    }
    if (done) return;
    const int r0 = lb * blockDim.x + threadIdx.x;
    const int stride = nbk * blockDim.x;
    constexpr int NV = FIRST ? 1 : 4;
    const T* src[NV];
    if constexpr (FIRST) {
        src[0] = V.r;
    } else {
        src[0] = V.s;
        src[1] = V.t;
        src[2] = V.p_old;
        src[3] = V.v_old;
    }
    RowRaw<B, T, NV> R;
    if (r0 < nA) fetch_row<B, T, NV>(ls, At, r0, src, R);
    block_sum<4>(red);
    double om = 0.0, rho, beta = 0.0;
    if (FIRST) {
        rho = red[0];                       // (rh, r_0) = |b~|^2
    } else {
        om = (red[1] > 0.0) ? red[0] / red[1] : 0.0;
        rho = red[2] - om * red[3];
        beta = (rho / rho_prev) * (al_prev / om);
    }
    const bool stop = !FIRST && (it >= S.maxit || om == 0.0 || !isfinite(beta));
    if (lb == 0 && threadIdx.x == 0) {
        sc->rho_hist[it & 1] = rho;
        sc->omega = om;
        sc->iters = it;      // iterations completed (x_it is formed here)
        if (stop) {
            sc->done = 1;
            sc->breakdown = 1;
        }
    }
    double dot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = r0; r < nA; r += stride) {
        if (r != r0) fetch_row<B, T, NV>(ls, At, r, src, R);
        double ri[B], pi[B], vi[B];
        if (FIRST) {
#pragma unroll
            for (int c = 0; c < B; c++) ri[c] = (double)R.xo[0][c];
        } else {
            // tail of iteration i-1 on the own row
#pragma unroll
            for (int c = 0; c < B; c++) {
                const long q = (long)r * B + c;
                const double sv = (double)R.xo[0][c];
                V.x[q] = (T)((double)V.x[q] + al_prev * (double)R.xo[2][c] + om * sv);
                ri[c] = (double)(T)(sv - om * (double)R.xo[1][c]);
                V.r[q] = (T)ri[c];
            }
        }
        if (stop) continue;
        auto fx = [&](const T (&raw)[NV][B], double (&x)[B]) {
#pragma unroll
            for (int c = 0; c < B; c++) {
                if constexpr (FIRST) {
                    x[c] = (double)raw[0][c];
                } else {
                    const double rr_ = (double)(T)((double)raw[0][c] - om * (double)raw[1][c]);
                    x[c] = (double)(T)(rr_ + beta * ((double)raw[2][c] - om * (double)raw[3][c]));
                }
            }
        };
        fx(R.xo, pi);
#pragma unroll
        for (int c = 0; c < B; c++) vi[c] = pi[c];
        finish_row<B, T, NV>(ls, At, src, R, vi, fx);
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            V.p_new[q] = (T)pi[c];
            const T vT = (T)vi[c];
            V.v_new[q] = vT;
            dot[0] += (double)V.rh[q] * (double)vT;
            dot[1] += (double)vT * (double)vT;
            dot[2] += ri[c] * ri[c];
        }
    }
    block_sum<4>(dot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) pa[4 * lb + k] = dot[k];
    }
}

// ------------------------------------------------------ kernel S (iter i)
// start: sigma = (rh, v_i), |v_i|^2, |r_i|^2 from kernel P.  Stops when
// |r_i|^2 <= tol2 (x_i is the answer) or on a breakdown of sigma; else
// alpha = rho_i / sigma, s = r_i - alpha v_i, t = A~ s (s rebuilt at the
// neighbours).  Partial sums: (t,s), (t,t), (rh,s), (rh,t).
template <int B, typename T>
__global__ __launch_bounds__(KB_NT) void k_bicg_s(const KSeg* __restrict__ segs,
                                                  const int* __restrict__ blk_seg, int it) {
    const KSeg& S = segs[blk_seg[blockIdx.x]];
    if (!S.active) return;
    const int lb = blockIdx.x - S.blk0, nbk = S.nblk, nA = S.nA;
    const LocalSys& ls = S.ls;
    const T* __restrict__ At = (const T*)S.kb.At;
    const Vecs<B, T> V = make_vecs<B, T>(S.kb, it & 1);
    KScal* __restrict__ sc = S.kb.sc;
    const double* __restrict__ pa = S.kb.part_a;
    double* __restrict__ pb = S.kb.part_b;
    const double brk = sizeof(T) == 4 ? 1e-6 : 1e-14;
    const int done = sc->done;
    const double rho = sc->rho_hist[it & 1];
    double red[3] = {0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nbk; q += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 3; k++) red[k] += pa[(long)q * 4 + k];
    }
    if (done) return;
    const T* const src[2] = {V.r, V.v_new};
    const int r0 = lb * blockDim.x + threadIdx.x;
    const int stride = nbk * blockDim.x;
    RowRaw<B, T, 2> R;
    if (r0 < nA) fetch_row<B, T, 2>(ls, At, r0, src, R);
    block_sum<3>(red);
    const double sigma = red[0], vv = red[1], rr = red[2];
    const double al = rho / sigma;
    const bool conv = rr <= S.tol2;
    const bool bad = !conv && (!(sigma * sigma > brk * brk * S.bnorm2 * vv) || !isfinite(al) ||
                               !isfinite(rr));
    if (lb == 0 && threadIdx.x == 0) {
        sc->rr = rr;
        if (conv || bad) {
            sc->done = 1;
            sc->iters = it;
            sc->breakdown = bad ? 1 : 0;
        } else {
            sc->alpha = al;
        }
    }
    if (conv || bad) return;
    auto fx = [&](const T (&raw)[2][B], double (&x)[B]) {
#pragma unroll
        for (int c = 0; c < B; c++) x[c] = s_update<T>(raw[0][c], raw[1][c], al);
    };
    double dot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = r0; r < nA; r += stride) {
        if (r != r0) fetch_row<B, T, 2>(ls, At, r, src, R);
        double si[B], ti[B];
        fx(R.xo, si);
#pragma unroll
        for (int c = 0; c < B; c++) ti[c] = si[c];
        finish_row<B, T, 2>(ls, At, src, R, ti, fx);
#pragma unroll
        for (int c = 0; c < B; c++) {
            const long q = (long)r * B + c;
            const T sT = (T)si[c], tT = (T)ti[c];
            V.s[q] = sT;
            V.t[q] = tT;
            const double h = (double)V.rh[q];
            dot[0] += (double)tT * (double)sT;
            dot[1] += (double)tT * (double)tT;
            dot[2] += h * (double)sT;
            dot[3] += h * (double)tT;
        }
    }
    block_sum<4>(dot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) pb[4 * lb + k] = dot[k];
    }
}

template <int B, typename T>
__global__ __launch_bounds__(KB_NT) void k_ir_accumulate(const KSeg* __restrict__ segs,
                                                         const int* __restrict__ blk_seg) {
    const KSeg& S = segs[blk_seg[blockIdx.x]];
    if (!S.active) return;
    const int lb = blockIdx.x - S.blk0, nbk = S.nblk;
    double* __restrict__ x64 = S.kb.x64;
    const T* __restrict__ xT = (const T*)S.kb.x;
    for (long q = (long)lb * blockDim.x + threadIdx.x; q < (long)S.nA * B;
         q += (long)nbk * blockDim.x)
        x64[q] += (double)xT[q];
}

__global__ void k_copy_f64(double* __restrict__ d, const double* __restrict__ s, long n) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) d[q] = s[q];
}

void launch_copy_f64(double* dst, const double* src, long n, hipStream_t s) {
    if (n > 0) k_copy_f64<<<nblocks(n), NT, 0, s>>>(dst, src, n);
}

// ------------------------------------------------------------- launches

// ev0/ev1 (optional): events stamped by the dispatch itself
// (hipExtLaunchKernelGGL), i.e. the kernel's own start and end
template <int B, typename T>
static void part_impl(int which, const KSeg* segs, const int* blk_seg, int nblk_total, int it,
                      hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 nb(nblk_total), nt(KB_NT);
    if (which == 0) {
        if (it == 0)
            hipExtLaunchKernelGGL(k_bicg_p<B, T, true>, nb, nt, 0, s, ev0, ev1, 0, segs, blk_seg, it);
        else
            hipExtLaunchKernelGGL(k_bicg_p<B, T, false>, nb, nt, 0, s, ev0, ev1, 0, segs, blk_seg, it);
    } else {
        hipExtLaunchKernelGGL(k_bicg_s<B, T>, nb, nt, 0, s, ev0, ev1, 0, segs, blk_seg, it);
    }
}

int krylov_grid(int nA) { return kgrid(nA); }

// One wave per model: Krylov status and the fixed-order sums of the
// refinement partials (|r64|^2, |b~|^2) of that model.
__global__ __launch_bounds__(64) void k_seg_status(const KSeg* __restrict__ segs, int nseg,
                                                   SegStatus* __restrict__ out) {
    const int k = blockIdx.x;
    if (k >= nseg) return;
    const KSeg& S = segs[k];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < S.nblk; q += 64) {
        a += S.kb.part_ir[2 * q];
        b += S.kb.part_ir[2 * q + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x == 0) {
        SegStatus o;
        o.rir2 = a;
        o.bnorm2 = b;
        o.done = S.kb.sc->done;
        o.iters = S.kb.sc->iters;
        o.breakdown = S.kb.sc->breakdown;
        o.pad = 0;
        out[k] = o;
    }
}

void launch_seg_status(const KSeg* segs, int nseg, SegStatus* out, hipStream_t s) {
    if (nseg > 0) k_seg_status<<<nseg, 64, 0, s>>>(segs, nseg, out);
}

#define KDISPATCH(MACRO)                                                        \
    if (fp32) {                                                                 \
        if (b == 1) MACRO(1, float); else if (b == 2) MACRO(2, float); else MACRO(3, float);      \
    } else {                                                                    \
        if (b == 1) MACRO(1, double); else if (b == 2) MACRO(2, double); else MACRO(3, double);   \
    }

void launch_ir_residual(int b, bool fp32, const KSeg* segs, const int* blk_seg, int nblk_total,
                        bool x_zero, hipStream_t s) {
    if (nblk_total <= 0) return;
#define IR(BV, TT) k_ir_residual<BV, TT><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg, x_zero ? 1 : 0)
    KDISPATCH(IR)
#undef IR
}

void launch_bicg_part(int which, int b, bool fp32, const KSeg* segs, const int* blk_seg,
                      int nblk_total, int it, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (nblk_total <= 0) return;
#define PI(BV, TT) part_impl<BV, TT>(which, segs, blk_seg, nblk_total, it, s, ev0, ev1)
    KDISPATCH(PI)
#undef PI
}

void launch_ir_accumulate(int b, bool fp32, const KSeg* segs, const int* blk_seg,
                          int nblk_total, hipStream_t s) {
    if (nblk_total <= 0) return;
#define AC(BV, TT) k_ir_accumulate<BV, TT><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg)
    KDISPATCH(AC)
#undef AC
}

} // namespace fimk
