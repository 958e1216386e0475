// Residual and Jacobian assembly on the active rows (Appendix A residual;
// J_A = R_A J R_A^T built directly, Section 4.3), the block-Jacobi
// scaling of the local system and the per-cell residual error measure of
// the residual-based localization.
//
// One thread per active row.  The row gathers every connection of its
// cell (an inactive neighbour contributes its frozen state: the Dirichlet
// condition of the local subproblem) and writes the off-diagonal block only
// for active neighbours.  Each connection is evaluated from both sides with
// the same canonical orientation (lower index first), so the two rows see
// bitwise-identical potential differences and upwind choices and the
// fluxes cancel exactly in the mass balance.  No atomics.
#include "fim_device.hpp"
#include "fim_physics.hpp"

namespace fimk {

template <int FK>
__global__ __launch_bounds__(NT) void k_accumulation(int n, const double* __restrict__ u,
                                                     const int8_t* __restrict__ st,
                                                     Graph g, DevFluid f,
                                                     double* __restrict__ M) {
    constexpr int B = FluidTraits<FK>::B;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double uu[B];
#pragma unroll
    for (int v = 0; v < B; v++) uu[v] = u[(long)v * n + i];
    Props<FK> P;
    cell_props<FK>(uu, st[i], g.pv[i], f, P);
#pragma unroll
    for (int c = 0; c < B; c++) M[(long)c * n + i] = P.M[c].v;
}

// batched timestep start (cell launch): copy of the state, accumulation at
// it (the same arithmetic as k_accumulation) and the first active flags
template <int FK>
__global__ __launch_bounds__(NT) void k_begin_seg(const BMember* __restrict__ t,
                                                  const BMap* __restrict__ map) {
    constexpr int B = FluidTraits<FK>::B;
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    const int n = M.n, i = e.vb * NT + threadIdx.x;
    if (!M.begin || i >= n) return;
    double uu[B];
#pragma unroll
    for (int v = 0; v < B; v++) {
        uu[v] = M.u[(long)v * n + i];
        M.un[(long)v * n + i] = uu[v];
    }
    const int8_t s = M.st[i];
    M.stn[i] = s;
    Props<FK> P;
    cell_props<FK>(uu, s, M.g.pv[i], M.f, P);
#pragma unroll
    for (int c = 0; c < B; c++) M.Mn[(long)c * n + i] = P.M[c].v;
    if (M.begin == 1) {
        M.act[i] = M.supp[i];
    } else if (M.begin == 2) {
        const bool seed = (M.g.flags[i] & CF_AA) != 0;
        M.lvl[i] = seed ? 0 : 0xff;
        M.act[i] = seed ? 1 : 0;
    } else if (M.begin == 3) {
        M.act[i] = 1;
    }
}

void launch_begin_seg(int fk, const BMember* t, const BMap* cells, int ncells, int layers,
                      hipStream_t s) {
    if (ncells <= 0) return;
    switch (fk) {
    case 1: k_begin_seg<1><<<ncells, NT, 0, s>>>(t, cells); break;
    case 2: k_begin_seg<2><<<ncells, NT, 0, s>>>(t, cells); break;
    default: k_begin_seg<3><<<ncells, NT, 0, s>>>(t, cells); break;
    }
    launch_ball_steps_seg(t, cells, ncells, layers, s);
}

// (vb: the workgroup's index among the NT-row workgroups of this system)
template <int FK>
__device__ inline void assemble_rows(int nA, const LocalSys& ls, const Graph& g,
                                     const DevFluid& f, const double* __restrict__ u,
                                     const int8_t* __restrict__ st,
                                     const double* __restrict__ Mn, double inv_dt, int vb) {
    constexpr int B = FluidTraits<FK>::B;
    constexpr int NPH = FluidTraits<FK>::NPH;
    constexpr int BB = B * B;
    const int r = vb * NT + threadIdx.x;
    if (r >= nA) return;
    const int n = g.n;
    const int i = ls.l2g[r];
    const long base = slot_of(ls, r, 0);   // slot k at base + 64 k
    const int width = ls.swidth[r / SLICE];

    double ui[B];
#pragma unroll
    for (int v = 0; v < B; v++) ui[v] = u[(long)v * n + i];
    Props<FK> Pi;
    cell_props<FK>(ui, st[i], g.pv[i], f, Pi);

    double R[B], Jd[B][B];
#pragma unroll
    for (int c = 0; c < B; c++) {
        R[c] = (Pi.M[c].v - Mn[(long)c * n + i]) * inv_dt;
#pragma unroll
        for (int v = 0; v < B; v++) Jd[c][v] = Pi.M[c].d[v] * inv_dt;
    }
    const double zi = g.depth[i];
    const double gg = f.gravity;
    int k = 1;
    const int e0 = g.adj_ptr[i], e1 = g.adj_ptr[i + 1];
    for (int e = e0; e < e1; e++) {
        const int j = g.adj_nbr[e];
        const double T = g.adj_T[e];
        const int lj = ls.g2l[j];
        double uj[B];
#pragma unroll
        for (int v = 0; v < B; v++) uj[v] = u[(long)v * n + j];
        Props<FK> Pj;
        cell_props<FK>(uj, st[j], g.pv[j], f, Pj);
        const double zj = g.depth[j];
        // canonical orientation: lo = lower index; flux f flows hi -> lo
        const bool i_lo = i < j;
        const double sgn = i_lo ? -1.0 : 1.0;   // R_i += sgn * f
        const double p_lo = i_lo ? ui[0] : uj[0];
        const double p_hi = i_lo ? uj[0] : ui[0];
        const double dz = i_lo ? (zj - zi) : (zi - zj);   // z_hi - z_lo
        double Jo[B][B];
#pragma unroll
        for (int c = 0; c < B; c++)
#pragma unroll
            for (int v = 0; v < B; v++) Jo[c][v] = 0.0;
#pragma unroll
        for (int l = 0; l < NPH; l++) {
            const Dual<B>& rlo = i_lo ? Pi.rho[l] : Pj.rho[l];
            const Dual<B>& rhi = i_lo ? Pj.rho[l] : Pi.rho[l];
            const double dphi = (p_hi - p_lo) - 0.5 * (rlo.v + rhi.v) * gg * dz;
            // d(dphi)/du_i and d(dphi)/du_j
            double ddi[B], ddj[B];
            const double gw = 0.5 * gg * dz;
#pragma unroll
            for (int v = 0; v < B; v++) {
                ddi[v] = -gw * Pi.rho[l].d[v];
                ddj[v] = -gw * Pj.rho[l].d[v];
            }
            ddi[0] += i_lo ? -1.0 : 1.0;
            ddj[0] += i_lo ? 1.0 : -1.0;
            const bool up_hi = dphi > 0.0;
            const bool up_i = (up_hi != i_lo);   // upstream cell is i
#pragma unroll
            for (int c = 0; c < B; c++) {
                if (!carries<FK>(c, l)) continue;
                const Dual<B>& mu_ = up_i ? Pi.mob[c][l] : Pj.mob[c][l];
                const double fl = T * mu_.v * dphi;
                R[c] += sgn * fl;
#pragma unroll
                for (int v = 0; v < B; v++) {
                    double di = T * mu_.v * ddi[v];
                    double dj = T * mu_.v * ddj[v];
                    if (up_i) di += T * mu_.d[v] * dphi;
                    else dj += T * mu_.d[v] * dphi;
                    Jd[c][v] += sgn * di;
                    Jo[c][v] += sgn * dj;
                }
            }
        }
        if (lj >= 0) {
            const long pos = base + (long)k * SLICE;
            ls.col[pos] = lj;
            double* out = ls.J + pos * BB;
#pragma unroll
            for (int c = 0; c < B; c++)
#pragma unroll
                for (int v = 0; v < B; v++) out[c * B + v] = Jo[c][v];
            k++;
        }
    }
    if (g.flags[i] & CF_PERF) {
        const double wi = g.wi[i];
        const double dpw = g.bhp[i] - ui[0];
#pragma unroll
        for (int c = 0; c < B; c++) {
            Dual<B> ms = dconst<B>(0.0);
#pragma unroll
            for (int l = 0; l < NPH; l++)
                if (carries<FK>(c, l)) ms = ms + Pi.mob[c][l];
            R[c] -= wi * ms.v * dpw;
#pragma unroll
            for (int v = 0; v < B; v++) Jd[c][v] -= wi * ms.d[v] * dpw;
            Jd[c][0] += wi * ms.v;
        }
    }
    // diagonal block and residual
    {
        const long pos = base;
        ls.col[pos] = r;
        double* out = ls.J + pos * BB;
#pragma unroll
        for (int c = 0; c < B; c++)
#pragma unroll
            for (int v = 0; v < B; v++) out[c * B + v] = Jd[c][v];
    }
    // padding slots up to the slice width: column = the row itself, no
    // block (readers of J recognise them by that column; k_precond writes
    // the zero blocks the FP64 product kernels load)
    for (; k < width; k++) ls.col[base + (long)k * SLICE] = r;
#pragma unroll
    for (int c = 0; c < B; c++) ls.F[(long)r * B + c] = R[c];
}

// ---------------------------------------------------------------------
// Error measure of the residual-based localization (the estimator of Lu
// and Beckner that Sections 1 and 4.2 describe), on every cell:
//     e_i = dt max_c |R_{i,c}| / (V_i rho_c)
// with R the residual of the Appendix A equations at the current state,
// V_i the reference pore volume and rho_c the reference density of
// component c: the step's mass imbalance of the cell as a fraction of its
// pore volume filled with that component.  The flux arithmetic (canonical
// orientation, phase-potential upwinding, well term) is that of k_assemble
// without the derivatives.
template <int FK>
__global__ __launch_bounds__(NT) void k_assemble(int nA, LocalSys ls, Graph g, DevFluid f,
                                                 const double* __restrict__ u,
                                                 const int8_t* __restrict__ st,
                                                 const double* __restrict__ Mn,
                                                 double inv_dt) {
    assemble_rows<FK>(nA, ls, g, f, u, st, Mn, inv_dt, blockIdx.x);
}

template <int FK>
__global__ __launch_bounds__(NT) void k_assemble_seg(const BMember* __restrict__ t,
                                                     const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    assemble_rows<FK>(M.nA, M.ls, M.g, M.f, M.u, M.st, M.Mn, M.inv_dt, e.vb);
}

template <int FK>
__device__ inline double ref_density(const DevFluid& f, int c) {
    if constexpr (FK == 1) return f.rho_ref;
    else if constexpr (FK == 2) return c == 0 ? f.rho_w : f.rho_o;
    else return c == 0 ? f.rho_wsc : (c == 1 ? f.rho_osc : f.rho_gsc);
}

template <int FK>
__device__ inline void resid_err_cells(int n, const Graph& g, const DevFluid& f,
                                       const double* __restrict__ u,
                                       const int8_t* __restrict__ st,
                                       const double* __restrict__ Mn, double dt,
                                       double* __restrict__ err, int vb) {
    constexpr int B = FluidTraits<FK>::B;
    constexpr int NPH = FluidTraits<FK>::NPH;
    const int i = vb * NT + threadIdx.x;
    if (i >= n) return;
    const double inv_dt = 1.0 / dt;
    double ui[B];
#pragma unroll
    for (int v = 0; v < B; v++) ui[v] = u[(long)v * n + i];
    Props<FK> Pi;
    cell_props<FK>(ui, st[i], g.pv[i], f, Pi);
    double R[B];
#pragma unroll
    for (int c = 0; c < B; c++) R[c] = (Pi.M[c].v - Mn[(long)c * n + i]) * inv_dt;
    const double zi = g.depth[i];
    const double gg = f.gravity;
    for (int e = g.adj_ptr[i]; e < g.adj_ptr[i + 1]; e++) {
        const int j = g.adj_nbr[e];
        const double T = g.adj_T[e];
        double uj[B];
#pragma unroll
        for (int v = 0; v < B; v++) uj[v] = u[(long)v * n + j];
        Props<FK> Pj;
        cell_props<FK>(uj, st[j], g.pv[j], f, Pj);
        const double zj = g.depth[j];
        const bool i_lo = i < j;
        const double sgn = i_lo ? -1.0 : 1.0;
        const double p_lo = i_lo ? ui[0] : uj[0];
        const double p_hi = i_lo ? uj[0] : ui[0];
        const double dz = i_lo ? (zj - zi) : (zi - zj);
#pragma unroll
        for (int l = 0; l < NPH; l++) {
            const double rlo = i_lo ? Pi.rho[l].v : Pj.rho[l].v;
            const double rhi = i_lo ? Pj.rho[l].v : Pi.rho[l].v;
            const double dphi = (p_hi - p_lo) - 0.5 * (rlo + rhi) * gg * dz;
            const bool up_i = ((dphi > 0.0) != i_lo);
#pragma unroll
            for (int c = 0; c < B; c++) {
                if (!carries<FK>(c, l)) continue;
                const double mob = up_i ? Pi.mob[c][l].v : Pj.mob[c][l].v;
                R[c] += sgn * (T * mob * dphi);
            }
        }
    }
    if (g.flags[i] & CF_PERF) {
        const double dpw = g.bhp[i] - ui[0];
#pragma unroll
        for (int c = 0; c < B; c++) {
            double ms = 0.0;
#pragma unroll
            for (int l = 0; l < NPH; l++)
                if (carries<FK>(c, l)) ms += Pi.mob[c][l].v;
            R[c] -= g.wi[i] * ms * dpw;
        }
    }
    double e = 0.0;
#pragma unroll
    for (int c = 0; c < B; c++) e = fmax(e, fabs(R[c]) / (g.pv[i] * ref_density<FK>(f, c)));
    err[i] = dt * e;
}

template <int FK>
__global__ __launch_bounds__(NT) void k_resid_err(int n, Graph g, DevFluid f,
                                                  const double* __restrict__ u,
                                                  const int8_t* __restrict__ st,
                                                  const double* __restrict__ Mn, double dt,
                                                  double* __restrict__ err) {
    resid_err_cells<FK>(n, g, f, u, st, Mn, dt, err, blockIdx.x);
}

// the error measure of the FIM_RESID members (cell launch)
template <int FK>
__global__ __launch_bounds__(NT) void k_resid_err_seg(const BMember* __restrict__ t,
                                                      const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode != FIM_RESID) return;
    resid_err_cells<FK>(M.n, M.g, M.f, M.u, M.st, M.Mn, M.dt, M.last_dp, e.vb);
}

// ---------------------------------------------------------------------
// Block-Jacobi scaling: dinv = (J_ii)^{-1} (FP64) and the scaled blocks
// A~_ik = dinv J_ik stored in the Krylov precision (the scaled diagonal is
// the identity and is not stored).
template <int B>
__device__ inline bool invert_block(const double* a, double* inv) {
    if constexpr (B == 1) {
        inv[0] = 1.0 / a[0];
        return a[0] != 0.0;
    } else if constexpr (B == 2) {
        const double det = a[0] * a[3] - a[1] * a[2];
        const double id = 1.0 / det;
        inv[0] = a[3] * id;
        inv[1] = -a[1] * id;
        inv[2] = -a[2] * id;
        inv[3] = a[0] * id;
        return det != 0.0;
    } else {
        // Gauss-Jordan with partial pivoting
        double m[B][2 * B];
#pragma unroll
        for (int r = 0; r < B; r++)
#pragma unroll
            for (int c = 0; c < B; c++) {
                m[r][c] = a[r * B + c];
                m[r][B + c] = (r == c) ? 1.0 : 0.0;
            }
        bool ok = true;
#pragma unroll
        for (int c = 0; c < B; c++) {
            int piv = c;
            double best = fabs(m[c][c]);
#pragma unroll
            for (int r = c + 1; r < B; r++)
                if (fabs(m[r][c]) > best) { best = fabs(m[r][c]); piv = r; }
            if (best == 0.0) ok = false;
            // row swap c <-> piv with compile-time indices only (a
            // runtime row index would put m in scratch memory)
#pragma unroll
            for (int q = 0; q < 2 * B; q++) {
                const double t0 = m[c][q];
                double tp = t0;
#pragma unroll
                for (int r = c + 1; r < B; r++)
                    if (piv == r) tp = m[r][q];
#pragma unroll
                for (int r = c + 1; r < B; r++)
                    if (piv == r) m[r][q] = t0;
                m[c][q] = tp;
            }
            const double ip = 1.0 / m[c][c];
#pragma unroll
            for (int q = 0; q < 2 * B; q++) m[c][q] *= ip;
#pragma unroll
            for (int r = 0; r < B; r++) {
                if (r == c) continue;
                const double fct = m[r][c];
#pragma unroll
                for (int q = 0; q < 2 * B; q++) m[r][q] -= fct * m[c][q];
            }
        }
#pragma unroll
        for (int r = 0; r < B; r++)
#pragma unroll
            for (int c = 0; c < B; c++) inv[r * B + c] = m[r][B + c];
        return ok;
    }
}

// (x64: when non-null, the row's initial guess is zeroed as well)
template <int B, typename T>
__device__ inline void precond_rows(int nA, const LocalSys& ls, double* __restrict__ dinv,
                                    T* __restrict__ At, double* __restrict__ x64, int vb) {
    constexpr int BB = B * B;
    const int r = vb * NT + threadIdx.x;
    if (r >= nA) return;
    if (x64) {
#pragma unroll
        for (int c = 0; c < B; c++) x64[(long)r * B + c] = 0.0;
    }
    const long base = slot_of(ls, r, 0);
    const int width = ls.swidth[r / SLICE];
    double d[BB], di[BB];
    const double* J = ls.J;
#pragma unroll
    for (int q = 0; q < BB; q++) d[q] = J[base * BB + q];
    invert_block<B>(d, di);
#pragma unroll
    for (int q = 0; q < BB; q++) dinv[(long)r * BB + q] = di[q];
    // UR slots at a time, their column words and blocks in one round of
    // loads.  Padding slots (column = the row itself past the diagonal)
    // have no block in J (what their J slots hold is never used): the FP64
    // product kernels load their A~ block, written here as zero; the FP32
    // ones and every other reader skip them by their column.
    constexpr int UR = 4;
    for (int k0 = 1; k0 < width; k0 += UR) {
        int cl[UR];
        double a[UR][BB];
#pragma unroll
        for (int u = 0; u < UR; u++) {
            const long pos = base + (long)min(k0 + u, width - 1) * SLICE;
            cl[u] = k0 + u < width ? ls.col[pos] : r;
#pragma unroll
            for (int q = 0; q < BB; q++) a[u][q] = J[pos * BB + q];
        }
#pragma unroll
        for (int u = 0; u < UR; u++) {
            if (k0 + u >= width) break;
            const long pos = base + (long)(k0 + u) * SLICE;
            const bool pad = cl[u] == r;
            if (pad && sizeof(T) == 4) continue;
#pragma unroll
            for (int rr = 0; rr < B; rr++)
#pragma unroll
                for (int cc = 0; cc < B; cc++) {
                    double acc = 0.0;
#pragma unroll
                    for (int t = 0; t < B; t++) acc += di[rr * B + t] * a[u][t * B + cc];
                    At[pos * BB + rr * B + cc] = pad ? (T)0 : (T)acc;
                }
        }
    }
}

template <int B, typename T>
__global__ __launch_bounds__(NT) void k_precond(int nA, LocalSys ls, double* __restrict__ dinv,
                                                T* __restrict__ At) {
    precond_rows<B, T>(nA, ls, dinv, At, nullptr, blockIdx.x);
}

template <int B, typename T>
__global__ __launch_bounds__(NT) void k_precond_seg(const BMember* __restrict__ t,
                                                    const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    precond_rows<B, T>(M.nA, M.ls, M.dinv, (T*)M.At, M.x64, e.vb);
}

// ------------------------------------------------------------- launches
void launch_accumulation(int fk, int n, const double* u, const int8_t* st,
                         const Graph& g, const DevFluid& f, double* M,
                         hipStream_t s) {
    if (n <= 0) return;
    const int nb = nblocks(n);
    switch (fk) {
    case 1: k_accumulation<1><<<nb, NT, 0, s>>>(n, u, st, g, f, M); break;
    case 2: k_accumulation<2><<<nb, NT, 0, s>>>(n, u, st, g, f, M); break;
    default: k_accumulation<3><<<nb, NT, 0, s>>>(n, u, st, g, f, M); break;
    }
}

void launch_assemble(int fk, int nA, const LocalSys& ls, const Graph& g,
                     const DevFluid& f, const double* u, const int8_t* st,
                     const double* Mn, double inv_dt, hipStream_t s) {
    if (nA <= 0) return;
    const int nb = nblocks(nA);
    switch (fk) {
    case 1: k_assemble<1><<<nb, NT, 0, s>>>(nA, ls, g, f, u, st, Mn, inv_dt); break;
    case 2: k_assemble<2><<<nb, NT, 0, s>>>(nA, ls, g, f, u, st, Mn, inv_dt); break;
    default: k_assemble<3><<<nb, NT, 0, s>>>(nA, ls, g, f, u, st, Mn, inv_dt); break;
    }
}

void launch_resid_err(int fk, int n, const Graph& g, const DevFluid& f, const double* u,
                      const int8_t* st, const double* Mn, double dt, double* err,
                      hipStream_t s) {
    if (n <= 0) return;
    const int nb = nblocks(n);
    switch (fk) {
    case 1: k_resid_err<1><<<nb, NT, 0, s>>>(n, g, f, u, st, Mn, dt, err); break;
    case 2: k_resid_err<2><<<nb, NT, 0, s>>>(n, g, f, u, st, Mn, dt, err); break;
    default: k_resid_err<3><<<nb, NT, 0, s>>>(n, g, f, u, st, Mn, dt, err); break;
    }
}

void launch_assemble_seg(int fk, const BMember* t, const BMap* rows, int nblk, hipStream_t s) {
    if (nblk <= 0) return;
    switch (fk) {
    case 1: k_assemble_seg<1><<<nblk, NT, 0, s>>>(t, rows); break;
    case 2: k_assemble_seg<2><<<nblk, NT, 0, s>>>(t, rows); break;
    default: k_assemble_seg<3><<<nblk, NT, 0, s>>>(t, rows); break;
    }
}

void launch_resid_err_seg(int fk, const BMember* t, const BMap* cells, int nblk, hipStream_t s) {
    if (nblk <= 0) return;
    switch (fk) {
    case 1: k_resid_err_seg<1><<<nblk, NT, 0, s>>>(t, cells); break;
    case 2: k_resid_err_seg<2><<<nblk, NT, 0, s>>>(t, cells); break;
    default: k_resid_err_seg<3><<<nblk, NT, 0, s>>>(t, cells); break;
    }
}

void launch_precond_seg(int b, bool fp32, const BMember* t, const BMap* rows, int nblk,
                        hipStream_t s) {
    if (nblk <= 0) return;
#define PC(BV, TT) k_precond_seg<BV, TT><<<nblk, NT, 0, s>>>(t, rows)
    if (fp32) {
        if (b == 1) PC(1, float); else if (b == 2) PC(2, float); else PC(3, float);
    } else {
        if (b == 1) PC(1, double); else if (b == 2) PC(2, double); else PC(3, double);
    }
#undef PC
}

void launch_precond(int b, bool fp32, int nA, const LocalSys& ls,
                    double* dinv, void* At, hipStream_t s) {
    if (nA <= 0) return;
    const int nb = nblocks(nA);
#define PC(BV, TT) k_precond<BV, TT><<<nb, NT, 0, s>>>(nA, ls, dinv, (TT*)At)
    if (fp32) {
        if (b == 1) PC(1, float); else if (b == 2) PC(2, float); else PC(3, float);
    } else {
        if (b == 1) PC(1, double); else if (b == 2) PC(2, double); else PC(3, double);
    }
#undef PC
}

} // namespace fimk
