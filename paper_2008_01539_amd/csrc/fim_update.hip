// Newton update u <- u + R_A^T du_A (Section 4.3), with the saturation chop,
// clamps and black-oil variable switching, the per-cell |dp| that drives
// the next active-set estimate, and the max-norms of the convergence test
// (Section 5: ||dp||_inf < eps_p).
#include "fim_device.hpp"
#include "fim_physics.hpp"

namespace fimk {

// owner (optional): only rows whose cell has owner[i] == own_k are
// updated (the additive form of Algorithm 2 combines overlapping subdomain
// updates by ownership); the others are left alone and do not count
// (vb: the workgroup's index among the system's NT-row workgroups; its
// partials go to part[4 vb ..])
template <int FK>
__device__ inline void update_rows(int nA, const int* __restrict__ l2g,
                                   const double* __restrict__ x64, double* __restrict__ u,
                                   int8_t* __restrict__ st, int n, const DevFluid& f,
                                   double ds_max, double* __restrict__ dp_abs,
                                   double* __restrict__ part, const int* __restrict__ owner,
                                   int own_k, int vb) {
    constexpr int B = FluidTraits<FK>::B;
    const int r = vb * NT + threadIdx.x;
    double red[4] = {0.0, 0.0, 0.0, 0.0};   // |dp| max, |dS| max, switches, nonfinite
    const int i = r < nA ? l2g[r] : 0;
    if (r < nA && (!owner || owner[i] == own_k)) {
        double du[B];
#pragma unroll
        for (int v = 0; v < B; v++) du[v] = x64[(long)r * B + v];
        int8_t status = (B == 3) ? st[i] : 0;
        if constexpr (B >= 2) {
            double sl = fabs(du[1]);
            if constexpr (B == 3) {
                if (status == 1) sl = fmax(sl, fabs(du[2]));
            }
            if (sl > ds_max) {
                const double sc = ds_max / sl;
                du[1] *= sc;
                if constexpr (B == 3) {
                    if (status == 1) du[2] *= sc;
                }
            }
        }
        double uu[B];
#pragma unroll
        for (int v = 0; v < B; v++) uu[v] = u[(long)v * n + i] + du[v];
        double dsm = 0.0;
        int nsw = 0;
        if constexpr (B >= 2) {
            dsm = fabs(du[1]);
            uu[1] = fmin(fmax(uu[1], 0.0), 1.0);
        }
        if constexpr (B == 3) {
            if (status == 1) {
                dsm = fmax(dsm, fabs(du[2]));
                uu[2] = fmin(uu[2], 1.0 - uu[1]);
            }
            const double rs_sat = f.rs_b * uu[0] / f.p_b;
            if (status == 1 && uu[2] < 0.0) {
                uu[2] = rs_sat;
                status = 0;
                nsw = 1;
            } else if (status == 0 && uu[2] > rs_sat) {
                uu[2] = 0.0;
                status = 1;
                nsw = 1;
            }
            st[i] = status;
        }
        bool finite = true;
#pragma unroll
        for (int v = 0; v < B; v++) {
            u[(long)v * n + i] = uu[v];
            finite = finite && isfinite(uu[v]);
        }
        const double dpa = fabs(du[0]);
        dp_abs[i] = dpa;
        red[0] = dpa;
        red[1] = dsm;
        red[2] = (double)nsw;
        red[3] = finite ? 0.0 : 1.0;
        if (!finite) red[0] = INFINITY;
    }
    block_max<2>(*reinterpret_cast<double(*)[2]>(&red[0]));
    block_sum<2>(*reinterpret_cast<double(*)[2]>(&red[2]));
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 4; q++) part[4 * vb + q] = red[q];
    }
}

template <int FK>
__global__ __launch_bounds__(NT) void k_update(int nA, const int* __restrict__ l2g,
                                               const double* __restrict__ x64,
                                               double* __restrict__ u, int8_t* __restrict__ st,
                                               int n, DevFluid f, double ds_max,
                                               double* __restrict__ dp_abs,
                                               double* __restrict__ part,
                                               const int* __restrict__ owner, int own_k) {
    update_rows<FK>(nA, l2g, x64, u, st, n, f, ds_max, dp_abs, part, owner, own_k, blockIdx.x);
}

template <int FK>
__global__ __launch_bounds__(NT) void k_update_seg(const BMember* __restrict__ t,
                                                   const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    update_rows<FK>(M.nA, M.ls.l2g, M.x64, M.u, M.st, M.n, M.f, M.ds_max, M.dp_abs, M.part,
                    nullptr, 0, e.vb);
}

// one block: combine the per-block maxima and counts of k_update
__device__ inline void update_finish(const double* __restrict__ part, int np, NStat* ns) {
    double mx[2] = {0.0, 0.0}, sm[2] = {0.0, 0.0};
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        mx[0] = fmax(mx[0], part[4 * q]);
        mx[1] = fmax(mx[1], part[4 * q + 1]);
        sm[0] += part[4 * q + 2];
        sm[1] += part[4 * q + 3];
    }
    block_max<2>(mx);
    block_sum<2>(sm);
    if (threadIdx.x == 0) {
        ns->dp_max = mx[0];
        ns->ds_max = mx[1];
        ns->nswitch = (int)sm[0];
        ns->nonfinite = (int)sm[1];
    }
}

__global__ __launch_bounds__(1024) void k_update_finish(const double* __restrict__ part, int np,
                                                        NStat* ns) {
    update_finish(part, np, ns);
}

// one block per member; also clears dint[0] for the set kernels that follow
__global__ __launch_bounds__(1024) void k_update_finish_seg(const BMember* __restrict__ t,
                                                            const BMap* __restrict__ map) {
    const BMember& M = t[map[blockIdx.x].q];
    update_finish(M.part, nblocks(M.nA > 0 ? M.nA : 1), M.ns);
    if (threadIdx.x == 0) M.dint[0] = 0;
}

void launch_update(int fk, int nA, const int* l2g, const double* x64,
                   double* u, int8_t* st, int n, const DevFluid& f,
                   double ds_max, double* dp_abs, double* part, NStat* ns,
                   hipStream_t s, const int* owner, int own_k) {
    const int nb = nblocks(nA > 0 ? nA : 1);
    switch (fk) {
    case 1: k_update<1><<<nb, NT, 0, s>>>(nA, l2g, x64, u, st, n, f, ds_max, dp_abs, part, owner, own_k); break;
    case 2: k_update<2><<<nb, NT, 0, s>>>(nA, l2g, x64, u, st, n, f, ds_max, dp_abs, part, owner, own_k); break;
    default: k_update<3><<<nb, NT, 0, s>>>(nA, l2g, x64, u, st, n, f, ds_max, dp_abs, part, owner, own_k); break;
    }
    k_update_finish<<<1, 1024, 0, s>>>(part, nb, ns);
}

void launch_update_seg(int fk, const BMember* t, const BMap* rows, int nblk, const BMap* mem,
                       int nmem, hipStream_t s) {
    if (nblk <= 0 || nmem <= 0) return;
    switch (fk) {
    case 1: k_update_seg<1><<<nblk, NT, 0, s>>>(t, rows); break;
    case 2: k_update_seg<2><<<nblk, NT, 0, s>>>(t, rows); break;
    default: k_update_seg<3><<<nblk, NT, 0, s>>>(t, rows); break;
    }
    k_update_finish_seg<<<nmem, 1024, 0, s>>>(t, mem);
}

__global__ void k_copy_state(int b, int n, const double* __restrict__ src,
                             const int8_t* __restrict__ ssrc, double* __restrict__ dst,
                             int8_t* __restrict__ sdst) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < (long)b * n) dst[q] = src[q];
    if (q < n) sdst[q] = ssrc[q];
}

void launch_copy_state(int b, int n, const double* src, const int8_t* ssrc,
                       double* dst, int8_t* sdst, hipStream_t s) {
    if (n > 0) k_copy_state<<<nblocks((long)b * n), NT, 0, s>>>(b, n, src, ssrc, dst, sdst);
}

} // namespace fimk
