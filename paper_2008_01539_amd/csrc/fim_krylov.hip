// Local linear solve J_A x = -F_A (Section 4.3; the paper does not name a
// linear solver).  BiCGStab on the block-Jacobi scaled system
// A~ = D^{-1} J_A (D = diagonal blocks) inside FP64 iterative refinement:
//
//   r64 = -F - J x64            (FP64, unscaled)
//   solve A~ d = D^{-1} r64     (BiCGStab in precision T: float or double)
//   x64 += d                    until ||r64|| <= lin_rtol ||F||.
//
// With fracture blocks (fim_fracpc.hip) BiCGStab runs on M^{-1} A~, M the
// block diagonal of A~ over fracture blocks: each product kernel applies
// M^{-1} to its tile's fracture rows before writing them (the blocks of a
// tile are local to its workgroup).
//
// One BiCGStab iteration is two kernels.  Each writes per-block partial
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
    // selects, not indexing: kb may be a kernel argument
    V.p_old = (T*)(parity ? kb.p[1] : kb.p[0]);
    V.v_old = (T*)(parity ? kb.v[1] : kb.v[0]);
    V.p_new = (T*)(parity ? kb.p[0] : kb.p[1]);
    V.v_new = (T*)(parity ? kb.v[0] : kb.v[1]);
    V.s = (T*)kb.sv;
    V.t = (T*)kb.t;
    return V;
}

// Loads and stores through the global address space with 32-bit byte
// offsets from a wave-uniform base: the compiler then issues global (not
// flat) memory instructions, which do not hold up LDS waits, and shares
// one offset register between arrays indexed alike.  Every array these
// kernels address this way stays below 4 GiB (checked at model creation).
#define FIM_GLOBAL __attribute__((address_space(1)))
template <typename V>
__device__ inline V ldg(const void* base, unsigned off) {
    return *(const FIM_GLOBAL V*)((const FIM_GLOBAL char*)base + off);
}
template <typename V>
__device__ inline void stg(void* base, unsigned off, V v) {
    *(FIM_GLOBAL V*)((FIM_GLOBAL char*)base + off) = v;
}
// N consecutive values of T at a byte offset, moved as vectors of up to 16
// bytes that are only T-aligned (dwordx2/x3/x4 memory instructions): one
// instruction per row vector instead of one per component.  Element-wise
// accesses through a 32-bit offset are not merged by the compiler (the
// offset arithmetic may wrap as far as it can tell).
template <typename T, int K>
using vec_of = T __attribute__((ext_vector_type(K), aligned(sizeof(T))));

template <int N, typename T>
__device__ inline void ldn(T* d, const void* base, unsigned off) {
    constexpr int K = (int)(16 / sizeof(T)) < N ? (int)(16 / sizeof(T)) : N;
    const vec_of<T, K> v = ldg<vec_of<T, K>>(base, off);
#pragma unroll
    for (int c = 0; c < K; c++) d[c] = v[c];
    if constexpr (N > K) ldn<N - K, T>(d + K, base, off + K * (unsigned)sizeof(T));
}
template <int N, typename T>
__device__ inline void stn(void* base, unsigned off, const T* d) {
    constexpr int K = (int)(16 / sizeof(T)) < N ? (int)(16 / sizeof(T)) : N;
    vec_of<T, K> v;
#pragma unroll
    for (int c = 0; c < K; c++) v[c] = d[c];
    stg<vec_of<T, K>>(base, off, v);
    if constexpr (N > K) stn<N - K, T>(base, off + K * (unsigned)sizeof(T), d + K);
}
template <int B, typename T>
__device__ inline void ldv(T (&d)[B], const void* base, unsigned off) {
    ldn<B, T>(d, base, off);
}
template <int B, typename T>
__device__ inline void stv(void* base, unsigned off, const T (&v)[B]) {
    stn<B, T>(base, off, v);
}

// Neighbour slots fetched together: enough to keep the raw operands of a
// chunk within about 104 VGPRs (column offsets, blocks and NV gathered
// vectors per slot), at most 8.
constexpr int CHUNK_BUDGET = 104;
template <int B, typename T, int NV, int BUDGET = CHUNK_BUDGET>
constexpr int chunk_slots() {
    constexpr int w = (int)sizeof(T) / 4;
    constexpr int per = 1 + (B * B + NV * B) * w;
    constexpr int u = BUDGET / per;
    return u < 2 ? 2 : (u > 8 ? 8 : u);
}

// Waves per SIMD the product kernels are compiled for (a VGPR cap of
// 512 / waves): three, except FP64 3x3 blocks, whose first chunk needs
// more registers than that leaves.
template <int B, typename T>
constexpr int kbp_waves() { return (B == 3 && sizeof(T) == 8) ? 2 : 3; }
// With the fracture-block step fused in (PC), two waves per SIMD; the WIDE
// FP32 variant runs three (smaller neighbour chunks, chunk_budget) so that
// systems of up to 3 x 64 x 4 x CUs rows take one pass of resident
// workgroups instead of a second, mostly idle one.
template <int B, typename T, int PC, bool WIDE>
constexpr int kb_waves() {
    return PC ? ((WIDE && sizeof(T) == 4) ? 3 : 2) : kbp_waves<B, T>();
}
template <typename T, int PC, bool WIDE>
constexpr int chunk_budget() { return (PC && WIDE && sizeof(T) == 4) ? 48 : CHUNK_BUDGET; }

// Slot geometry of row r: slot k at base + 64 k; width slots are in use
// (the slice's widest row; narrower rows are padded with column r and a
// zero block), cap (the slice stride) bounds the slots that may be read at
// all.
struct RowGeo {
    unsigned base, width, cap, row;
};
__device__ inline RowGeo row_geo(const LocalSys& ls, int r) {
    RowGeo g;
    g.base = (unsigned)slot_of(ls, r, 0);
    g.width = (unsigned)ldg<int>(ls.swidth, 4u * (unsigned)(r / SLICE));
    g.cap = (unsigned)ls.wcap;
    g.row = (unsigned)r;
    return g;
}

// The segment a block works on: the first of the table for a
// single-model launch (no block-to-model lookup in front of it), else
// looked up by block.
template <bool SOLO>
__device__ inline const KSeg& seg_of(const KSeg* segs, const int* blk_seg) {
    if constexpr (SOLO) return segs[0];
    else return segs[blk_seg[blockIdx.x]];
}

// Raw operands of U off-diagonal slots k0 .. k0+U-1 of one row: the blocks
// of A~ and the values of NV source vectors at the neighbours.  The column
// indices of every slot below the slice stride are loaded at once,
// together with the slice width (their addresses follow from the row index
// alone); the blocks and gathers of the slots below the width follow, so a
// chunk costs about two memory round trips.  Column words at or past the
// width (stale memory) are never used, and in FP32 padding slots (column =
// the row itself past the diagonal) load nothing: their block is zero.
template <int B, typename T, int NV, int U>
struct Chunk {
    T a[U][B * B];
    T xn[NV][U][B];
};

template <int B, typename T, int NV, int U>
__device__ inline void fetch_chunk(const LocalSys& ls, const T* At, const RowGeo& g, unsigned k0,
                                   const T* const (&src)[NV], Chunk<B, T, NV, U>& ch) {
    constexpr unsigned BB = B * B, RB = B * sizeof(T);
    unsigned cl[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const unsigned k = k0 + u;
        cl[u] = 0;
        if (k < g.cap) cl[u] = (unsigned)ldg<int>(ls.col, 4u * (g.base + k * SLICE));
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        const unsigned k = k0 + u;
        // (FP32 kernels only: the FP64 ones have no register left for it)
        const bool pad = sizeof(T) == 4 && cl[u] == g.row;
        if (k < g.width && !pad) {
            const unsigned ab = (g.base + k * SLICE) * (BB * (unsigned)sizeof(T));
            ldn<(int)BB, T>(ch.a[u], At, ab);
#pragma unroll
            for (int v = 0; v < NV; v++) ldv<B, T>(ch.xn[v][u], src[v], cl[u] * RB);
        } else {
#pragma unroll
            for (unsigned q = 0; q < BB; q++) ch.a[u][q] = (T)0;
#pragma unroll
            for (int v = 0; v < NV; v++)
#pragma unroll
                for (int c = 0; c < B; c++) ch.xn[v][u][c] = (T)0;
        }
    }
}

// y += sum over the chunk of A~_rk f(raw values at neighbour k), in FP64
template <int B, typename T, int NV, int U, class FX>
__device__ inline void apply_chunk(const Chunk<B, T, NV, U>& ch, unsigned k0, unsigned width,
                                   double (&y)[B], FX fx) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (k0 + u >= width) break;
        T raw[NV][B];
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int c = 0; c < B; c++) raw[v][c] = ch.xn[v][u][c];
        double xj[B];
        fx(raw, xj);
#pragma unroll
        for (int c = 0; c < B; c++) {
            double acc = 0.0;
#pragma unroll
            for (int v = 0; v < B; v++) acc += (double)ch.a[u][c * B + v] * xj[v];
            y[c] += acc;
        }
    }
}

// all off-diagonal slots of a row: the first chunk is already in ch (it
// was fetched early); wider rows reuse ch for the following chunks, so the
// operands of one chunk at a time are live
template <int B, typename T, int NV, int U, class FX>
__device__ inline void row_product(const LocalSys& ls, const T* At, const RowGeo& g,
                                   const T* const (&src)[NV], Chunk<B, T, NV, U>& ch,
                                   double (&y)[B], FX fx) {
#pragma unroll 1
    for (unsigned k0 = 1; k0 < g.width; k0 += U) {
        if (k0 > 1) fetch_chunk<B, T, NV, U>(ls, At, g, k0, src, ch);
        apply_chunk<B, T, NV, U>(ch, k0, g.width, y, fx);
    }
}

typedef float f4v __attribute__((ext_vector_type(4)));

// Left application of the fracture-block inverses inside the product
// kernels: y holds this thread's row of A~ x; rows of multi-row fracture
// blocks get the block's M^{-1} applied (the block's other rows are in the
// same tile, exchanged through LDS in the stored precision T, the values
// the unpreconditioned product would have written).  Every thread of the
// workgroup calls it; tiles without such blocks return after one barrier.
// The thread of block row rr reads its b rows of M^{-1} as 16-byte vectors
// (the grouped layout keeps them contiguous per group of K columns), 16
// columns per round with all loads of a round in flight together.  For
// b <= 2 the first round does not wait for the product: pc_first issues it
// before the row's product, pc_rows consumes it.
template <int B, typename T, bool DEC = false>
struct PcShape {
    static constexpr int K = pc_group_cols(B), W = B * K, NV4 = W / 4;
    // groups per round (decoupled blocks have b times fewer columns: two
    // groups per round keep the registers of the fused kernels)
    static constexpr int QG = DEC ? 2 : (B == 3 && sizeof(T) == 8) ? 2 : 16 / K;
    static constexpr bool PRE = B <= 2;                                   // first round early
};

template <int B, typename T, bool DEC = false>
using PcRound = f4v[PcShape<B, T, DEC>::QG][PcShape<B, T, DEC>::NV4];

// the inverse entries of round g0 of this thread's block row
template <int B, typename T, bool DEC>
__device__ inline void pc_load(const float* pcM, unsigned row0, unsigned grpb, int G, int g0,
                               PcRound<B, T, DEC>& mv) {
    using Sh = PcShape<B, T, DEC>;
#pragma unroll
    for (int q = 0; q < Sh::QG; q++) {
        const int gq = min(g0 + q, G - 1);
#pragma unroll
        for (int v = 0; v < Sh::NV4; v++) mv[q][v] = ldg<f4v>(pcM, row0 + (unsigned)gq * grpb + 16u * v);
    }
}

// first round of the row with layout words (info, off), if it is in a
// multi-row block (called with the row's tile pass current).  DEC: the
// block's unknowns decoupled (FIM_PC_FRACTURE): the layout's columns are
// the block's cells, and output c of a row takes unknown c of each cell.
template <int B, typename T, bool DEC>
__device__ inline void pc_first(const KrylovBufs& kb, int info, int off,
                                PcRound<B, T, DEC>& pm) {
    using Sh = PcShape<B, T, DEC>;
    if constexpr (Sh::PRE) {
        const int size = info & 0xffff;
        if (size > 1) {
            const int bs = info >> 16, ncol = DEC ? size : size * B;
            const unsigned row0 = (unsigned)(off + ((int)threadIdx.x - bs) * Sh::W) * 4u;
            pc_load<B, T, DEC>(kb.pcM, row0, (unsigned)(size * Sh::W) * 4u, (ncol + Sh::K - 1) / Sh::K,
                          0, pm);
        }
    }
}

template <int B, typename T, bool DEC>
__device__ inline void pc_rows(const KrylovBufs& kb, bool act, int info, int off,
                               double (&y)[B], const PcRound<B, T, DEC>& pm) {
    using Sh = PcShape<B, T, DEC>;
    constexpr int K = Sh::K, W = Sh::W, QG = Sh::QG;
    __shared__ T yb[KB_NT * B];
    const int t = threadIdx.x;
    const bool blk = act && (info & 0xffff) > 1;
    if (!__syncthreads_or(blk)) return;
    if (act) {
#pragma unroll
        for (int c = 0; c < B; c++) yb[t * B + c] = (T)y[c];
    }
    __syncthreads();
    if (blk) {
        const int size = info & 0xffff, bs = info >> 16, N = DEC ? size : size * B;
        const int G = (N + K - 1) / K;
        const unsigned row0 = (unsigned)(off + (t - bs) * W) * 4u;
        const unsigned grpb = (unsigned)(size * W) * 4u;
        const T* yv = yb + bs * B;
        double acc[B];
#pragma unroll
        for (int c = 0; c < B; c++) acc[c] = 0.0;
        auto round = [&](int g0, const PcRound<B, T, DEC>& mv) {
            if constexpr (!DEC) {
                T ys[QG][K];
#pragma unroll
                for (int q = 0; q < QG; q++) {
                    const int gq = min(g0 + q, G - 1);
#pragma unroll
                    for (int k = 0; k < K; k++) ys[q][k] = yv[min(gq * K + k, N - 1)];
                }
#pragma unroll
                for (int q = 0; q < QG; q++) {
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const int j = (g0 + q) * K + k;   // past N: padding or a clamped repeat
                        const double w = j < N ? (double)ys[q][k] : 0.0;
#pragma unroll
                        for (int c = 0; c < B; c++) {
                            const int e = c * K + k;
                            acc[c] += (double)mv[q][e / 4][e % 4] * w;
                        }
                    }
                }
            } else {
                // column j = cell j of the block: output c takes its unknown c
#pragma unroll
                for (int q = 0; q < QG; q++) {
                    const int gq = min(g0 + q, G - 1);
                    T ys[K][B];
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const int j = min(gq * K + k, N - 1);
#pragma unroll
                        for (int c = 0; c < B; c++) ys[k][c] = yv[j * B + c];
                    }
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const bool in = (g0 + q) * K + k < N;
#pragma unroll
                        for (int c = 0; c < B; c++) {
                            const int e = c * K + k;
                            acc[c] += (double)mv[q][e / 4][e % 4] * (in ? (double)ys[k][c] : 0.0);
                        }
                    }
                }
            }
        };
        int g0 = 0;
        if constexpr (Sh::PRE) {
            round(0, pm);
            g0 = QG;
        }
#pragma unroll 1
        for (; g0 < G; g0 += QG) {
            PcRound<B, T, DEC> mv;
            pc_load<B, T, DEC>(kb.pcM, row0, grpb, G, g0, mv);
            round(g0, mv);
        }
#pragma unroll
        for (int c = 0; c < B; c++) y[c] = acc[c];
    }
    __syncthreads();   // yb is reused by the next tile pass
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
template <int B, typename T, bool SOLO>
__global__ __launch_bounds__(KB_NT) void k_ir_residual(const KSeg* __restrict__ segs,
                                                       const int* __restrict__ blk_seg,
                                                       int x_zero) {
    const KSeg& S = seg_of<SOLO>(segs, blk_seg);
    if (!S.active) return;
    const int nbk = S.nblk, nA = S.nA, lb = xcd_tile(S.blk0, nbk, blockIdx.x);
    const LocalSys& ls = S.ls;
    const KrylovBufs& kb = S.kb;
    constexpr int BB = B * B;
    T* xT = (T*)kb.x;
    T* rr = (T*)kb.r;
    T* rh = (T*)kb.rh;
    double part[2] = {0.0, 0.0};
    const bool pc = kb.pcM != nullptr;
    // whole tiles per pass, so that the preconditioner's barriers are uniform
    for (int tb = lb * KB_NT; tb < nA; tb += nbk * KB_NT) {
        const int r = tb + threadIdx.x;
        const bool act = r < nA;
        double bt[B];
        int pinfo = 0, poff = 0;
#pragma unroll
        for (int c = 0; c < B; c++) bt[c] = 0.0;
        if (act) {
            double res[B];
#pragma unroll
            for (int c = 0; c < B; c++) res[c] = -ls.F[(long)r * B + c];
            if (!x_zero) {
                // UR slots at a time: their column indices in one round of
                // loads, then their FP64 blocks and x64 gathers in the next
                // (slots past the width, and padding slots, read no block:
                // weight 0); the slots are summed in order, as one at a time
                // would
                constexpr int UR = B == 3 ? 4 : 8;
                const long base = slot_of(ls, r, 0);
                const int width = ls.swidth[r / SLICE];
                for (int k0 = 0; k0 < width; k0 += UR) {
                    int cl[UR];
#pragma unroll
                    for (int u = 0; u < UR; u++)
                        cl[u] = k0 + u < width ? ls.col[base + (long)(k0 + u) * SLICE] : r;
                    double a[UR][BB], xv[UR][B];
#pragma unroll
                    for (int u = 0; u < UR; u++) {
                        // padding past the diagonal (column r) holds a zero block
                        const bool in = k0 + u < width && (k0 + u == 0 || cl[u] != r);
                        const long pos = base + (long)min(k0 + u, width - 1) * SLICE;
#pragma unroll
                        for (int q = 0; q < BB; q++) a[u][q] = in ? ls.J[pos * BB + q] : 0.0;
#pragma unroll
                        for (int v = 0; v < B; v++) xv[u][v] = kb.x64[(long)cl[u] * B + v];
                    }
#pragma unroll
                    for (int u = 0; u < UR; u++) {
                        if (k0 + u >= width) break;
#pragma unroll
                        for (int c = 0; c < B; c++) {
                            double acc = 0.0;
#pragma unroll
                            for (int v = 0; v < B; v++) acc += a[u][c * B + v] * xv[u][v];
                            res[c] -= acc;
                        }
                    }
                }
            }
            const double* di = kb.dinv + (long)r * BB;
#pragma unroll
            for (int c = 0; c < B; c++) {
                kb.rir[(long)r * B + c] = res[c];
                part[0] += res[c] * res[c];
                double s_ = 0.0;
#pragma unroll
                for (int v = 0; v < B; v++) s_ += di[c * B + v] * res[v];
                bt[c] = s_;
            }
            if (pc) {
                pinfo = kb.pcinfo[r];
                poff = kb.pcoff[r];
            }
        }
        if (pc && kb.pcdec) {
            PcRound<B, double, true> pm;
            if (act) pc_first<B, double, true>(kb, pinfo, poff, pm);
            pc_rows<B, double, true>(kb, act, pinfo, poff, bt, pm);
        } else if (pc) {
            PcRound<B, double, false> pm;
            if (act) pc_first<B, double, false>(kb, pinfo, poff, pm);
            pc_rows<B, double, false>(kb, act, pinfo, poff, bt, pm);
        }
        if (act) {
#pragma unroll
            for (int c = 0; c < B; c++) {
                const T btT = (T)bt[c];
                xT[(long)r * B + c] = (T)0;
                rr[(long)r * B + c] = btT;
                rh[(long)r * B + c] = btT;
                part[1] += (double)btT * (double)btT;
            }
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

__device__ inline void put_status(SegStatus* o, double rr, int done, int iters, int brk) {
    o->rir2 = 0.0;
    o->bnorm2 = 0.0;
    o->rr = rr;
    o->done = done;
    o->iters = iters;
    o->breakdown = brk;
    o->pad = 0;
}

// ------------------------------------------------------ kernel P (iter i)
// Finishes iteration i-1 and starts iteration i:
//   omega = (t,s)/(t,t), rho_i = (rh,s) - omega (rh,t)   [from kernel S]
//   x += alpha p + omega s;  r_i = s - omega t           [own rows]
//   p_i = r_i + beta (p_{i-1} - omega v_{i-1});  v_i = A~ p_i
// with p_i at the neighbours rebuilt from s, t, p, v on the fly (the same
// expression as on the own row, so both see the same value).  Vectors are
// stored in T; all arithmetic is FP64.
// Partial sums: (rh, v_i), (v_i, v_i), (r_i, r_i).  At i = 0, p_0 = r_0
// (the refinement initialisation) and x = 0 stays.  Stops (after the x, r
// update) at the iteration cap or when omega = 0.  The own-row operands
// and the first chunk of neighbour slots are fetched before the previous
// kernel's partial sums are reduced, so those loads overlap the reduction.
// PC: fracture blocks (0 none, 1 coupled, 2 the unknowns decoupled)
template <int B, typename T, bool FIRST, bool SOLO, int PC, bool WIDE>
__global__ __launch_bounds__(KB_NT, (kb_waves<B, T, PC, WIDE>())) void k_bicg_p(const KSeg* __restrict__ segs,
                                                                      const int* __restrict__ blk_seg,
                                                                      int it) {
    const KSeg& S = seg_of<SOLO>(segs, blk_seg);
    if (!S.active) return;
    const int nbk = S.nblk, nA = S.nA, lb = xcd_tile(S.blk0, nbk, blockIdx.x);
    const LocalSys& ls = S.ls;
    const T* At = (const T*)S.kb.At;
    const Vecs<B, T> V = make_vecs<B, T>(S.kb, it & 1);
    KScal* __restrict__ sc = S.kb.sc;
    const double* __restrict__ pin = FIRST ? S.kb.part_c : S.kb.part_b;
    double* __restrict__ pa = S.kb.part_a;
    const int done = sc->done;
    const double rho_prev = FIRST ? 1.0 : sc->rho_hist[(it - 1) & 1];
    const double al_prev = sc->alpha;
    constexpr int NR = FIRST ? 1 : 4;
    const bool pc = PC && S.kb.pcM != nullptr;   // uniform over the launch's segment
    double red[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nbk; q += blockDim.x) {
#pragma unroll
        for (int k = 0; k < NR; k++) red[k] += pin[(long)q * 4 + k];
    }
    if (done) return;
    const int r0 = lb * blockDim.x + threadIdx.x;
    const int stride = nbk * blockDim.x;
    constexpr int NV = FIRST ? 1 : 4;
    constexpr int U = chunk_slots<B, T, NV, chunk_budget<T, PC, WIDE>()>();
    constexpr unsigned RB = B * sizeof(T);
    const T* src[NV];
    if constexpr (FIRST) {
        src[0] = V.r;
    } else {
        src[0] = V.s;
        src[1] = V.t;
        src[2] = V.p_old;
        src[3] = V.v_old;
    }
    RowGeo g{0, 0, 0, 0};
    T own[NV][B] = {}, ox[B] = {}, orh[B] = {};
    Chunk<B, T, NV, U> ch{};
    int pinfo = 1, poff = 0;   // fracture-block layout of the row
    auto fetch = [&](int r) {
        g = row_geo(ls, r);
        const unsigned ro = (unsigned)r * RB;
#pragma unroll
        for (int v = 0; v < NV; v++) ldv<B, T>(own[v], src[v], ro);
        if constexpr (!FIRST) ldv<B, T>(ox, V.x, ro);
        ldv<B, T>(orh, V.rh, ro);
        if (pc) {
            pinfo = ldg<int>(S.kb.pcinfo, 4u * (unsigned)r);
            poff = ldg<int>(S.kb.pcoff, 4u * (unsigned)r);
        }
        fetch_chunk<B, T, NV, U>(ls, At, g, 1, src, ch);
    };
    if (r0 < nA) fetch(r0);
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
    // p_i from the raw (s, t, p_{i-1}, v_{i-1}) of a row: FP64 arithmetic,
    // r_i and p_i rounded to T as they are stored
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
    double dot[4] = {0.0, 0.0, 0.0, 0.0};
    // whole tiles per pass (r - threadIdx.x is the tile base), and the
    // fracture-block step outside every per-row branch: its barriers are
    // reached by all waves of the workgroup the same number of times
    for (int r = r0; r - (int)threadIdx.x < nA; r += stride) {
        const bool act = r < nA;
        const unsigned ro = (unsigned)r * RB;
        double vi[B];
#pragma unroll
        for (int c = 0; c < B; c++) vi[c] = 0.0;
        PcRound<B, T, PC == 2> pm;   // first round of the row's inverse entries
        if (act) {
            T ri[B];
            if constexpr (FIRST) {
#pragma unroll
                for (int c = 0; c < B; c++) ri[c] = own[0][c];
            } else {
                // tail of iteration i-1 on the own row
                T xn[B];
#pragma unroll
                for (int c = 0; c < B; c++) {
                    const double sv = (double)own[0][c];
                    xn[c] = (T)((double)ox[c] + al_prev * (double)own[2][c] + om * sv);
                    ri[c] = (T)(sv - om * (double)own[1][c]);
                }
                stv<B, T>(V.x, ro, xn);
                stv<B, T>(V.r, ro, ri);
            }
            if (!stop) {
                if (pc) pc_first<B, T, PC == 2>(S.kb, pinfo, poff, pm);
                double pi[B];
                fx(own, pi);
#pragma unroll
                for (int c = 0; c < B; c++) vi[c] = pi[c];      // diagonal block of A~ is I
                row_product<B, T, NV, U>(ls, At, g, src, ch, vi, fx);
                T pT[B];
#pragma unroll
                for (int c = 0; c < B; c++) {
                    pT[c] = (T)pi[c];
                    dot[2] += (double)ri[c] * (double)ri[c];
                }
                stv<B, T>(V.p_new, ro, pT);
            }
        }
        if (stop) {   // uniform: x and r only
            if (act && r + stride < nA) fetch(r + stride);
            continue;
        }
        if (pc) pc_rows<B, T, PC == 2>(S.kb, act, pinfo, poff, vi, pm);   // v = M^{-1} A~ p
        if (act) {
            T vT[B];
#pragma unroll
            for (int c = 0; c < B; c++) {
                vT[c] = (T)vi[c];
                dot[0] += (double)orh[c] * (double)vT[c];
                dot[1] += (double)vT[c] * (double)vT[c];
            }
            stv<B, T>(V.v_new, ro, vT);
            // (fetched here, not at the top of the loop, so that the first
            // chunk's registers are dead during the rest of the row)
            if (r + stride < nA) fetch(r + stride);
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
template <int B, typename T, bool SOLO, int PC, bool WIDE>
__global__ __launch_bounds__(KB_NT, (kb_waves<B, T, PC, WIDE>())) void k_bicg_s(const KSeg* __restrict__ segs,
                                                                      const int* __restrict__ blk_seg,
                                                                      int it,
                                                                      SegStatus* __restrict__ rec) {
    const KSeg& S = seg_of<SOLO>(segs, blk_seg);
    if (!S.active) return;
    const int nbk = S.nblk, nA = S.nA, lb = xcd_tile(S.blk0, nbk, blockIdx.x);
    const LocalSys& ls = S.ls;
    const T* At = (const T*)S.kb.At;
    const Vecs<B, T> V = make_vecs<B, T>(S.kb, it & 1);
    KScal* __restrict__ sc = S.kb.sc;
    const double* __restrict__ pa = S.kb.part_a;
    double* __restrict__ pb = S.kb.part_b;
    const double brk = sizeof(T) == 4 ? 1e-6 : 1e-14;
    const int done = sc->done;
    const double rho = sc->rho_hist[it & 1];
    const bool pc = PC && S.kb.pcM != nullptr;
    double red[3] = {0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nbk; q += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 3; k++) red[k] += pa[(long)q * 4 + k];
    }
    // rec (the last kernel S of a block of iterations): each model's
    // Krylov status after this kernel, for the host's check
    const int segi = SOLO ? 0 : blk_seg[blockIdx.x];
    if (done) {
        if (rec && lb == 0 && threadIdx.x == 0)
            put_status(rec + segi, sc->rr, 1, sc->iters, sc->breakdown);
        return;
    }
    constexpr int NV = 2;
    constexpr int U = chunk_slots<B, T, NV, chunk_budget<T, PC, WIDE>()>();
    constexpr unsigned RB = B * sizeof(T);
    const T* const src[NV] = {V.r, V.v_new};
    const int r0 = lb * blockDim.x + threadIdx.x;
    const int stride = nbk * blockDim.x;
    RowGeo g{0, 0, 0, 0};
    T own[NV][B] = {}, orh[B] = {};
    Chunk<B, T, NV, U> ch{};
    int pinfo = 1, poff = 0;   // fracture-block layout of the row
    auto fetch = [&](int r) {
        g = row_geo(ls, r);
        const unsigned ro = (unsigned)r * RB;
#pragma unroll
        for (int v = 0; v < NV; v++) ldv<B, T>(own[v], src[v], ro);
        ldv<B, T>(orh, V.rh, ro);
        if (pc) {
            pinfo = ldg<int>(S.kb.pcinfo, 4u * (unsigned)r);
            poff = ldg<int>(S.kb.pcoff, 4u * (unsigned)r);
        }
        fetch_chunk<B, T, NV, U>(ls, At, g, 1, src, ch);
    };
    if (r0 < nA) fetch(r0);
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
        if (rec) put_status(rec + segi, rr, (conv || bad) ? 1 : 0, it, bad ? 1 : 0);
    }
    if (conv || bad) return;
    auto fx = [&](const T (&raw)[NV][B], double (&x)[B]) {
#pragma unroll
        for (int c = 0; c < B; c++) x[c] = (double)(T)((double)raw[0][c] - al * (double)raw[1][c]);
    };
    double dot[4] = {0.0, 0.0, 0.0, 0.0};
    // whole tiles per pass, the fracture-block step outside every per-row
    // branch (its barriers are uniform over the workgroup)
    for (int r = r0; r - (int)threadIdx.x < nA; r += stride) {
        const bool act = r < nA;
        const unsigned ro = (unsigned)r * RB;
        double ti[B];
        T sT[B];
#pragma unroll
        for (int c = 0; c < B; c++) {
            ti[c] = 0.0;
            sT[c] = (T)0;
        }
        PcRound<B, T, PC == 2> pm;   // first round of the row's inverse entries
        if (act) {
            if (pc) pc_first<B, T, PC == 2>(S.kb, pinfo, poff, pm);
            double si[B];
            fx(own, si);
#pragma unroll
            for (int c = 0; c < B; c++) ti[c] = si[c];
            row_product<B, T, NV, U>(ls, At, g, src, ch, ti, fx);
#pragma unroll
            for (int c = 0; c < B; c++) {
                sT[c] = (T)si[c];
                dot[2] += (double)orh[c] * (double)sT[c];
            }
            stv<B, T>(V.s, ro, sT);
        }
        if (pc) pc_rows<B, T, PC == 2>(S.kb, act, pinfo, poff, ti, pm);   // t = M^{-1} A~ s
        if (act) {
            T tT[B];
#pragma unroll
            for (int c = 0; c < B; c++) {
                tT[c] = (T)ti[c];
                const double sd = (double)sT[c], td = (double)tT[c], h = (double)orh[c];
                dot[0] += td * sd;
                dot[1] += td * td;
                dot[3] += h * td;
            }
            stv<B, T>(V.t, ro, tT);
            if (r + stride < nA) fetch(r + stride);
        }
    }
    block_sum<4>(dot);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 4; k++) pb[4 * lb + k] = dot[k];
    }
}

template <int B, typename T, bool SOLO>
__global__ __launch_bounds__(KB_NT) void k_ir_accumulate(const KSeg* __restrict__ segs,
                                                         const int* __restrict__ blk_seg) {
    const KSeg& S = seg_of<SOLO>(segs, blk_seg);
    if (!S.active) return;
    const int nbk = S.nblk, lb = xcd_tile(S.blk0, nbk, blockIdx.x);
    double* __restrict__ x64 = S.kb.x64;
    const T* __restrict__ xT = (const T*)S.kb.x;
    // (an FP32 pass keeps the previous x64 in xprev, to be undone if the
    // pass stalls)
    double* __restrict__ xprev = S.kb.xprev;
    for (long q = (long)lb * blockDim.x + threadIdx.x; q < (long)S.nA * B;
         q += (long)nbk * blockDim.x) {
        const double o = x64[q];
        if (sizeof(T) == 4) xprev[q] = o;
        x64[q] = o + (double)xT[q];
    }
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
template <int B, typename T, bool SOLO, int PC, bool WIDE>
static void part_impl_w(int which, const KSeg* segs, const int* blk_seg, int nblk_total, int it,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, SegStatus* rec) {
    const dim3 nb(nblk_total), nt(KB_NT);
    if (which == 0) {
        if (it == 0)
            hipExtLaunchKernelGGL(k_bicg_p<B, T, true, SOLO, PC, WIDE>, nb, nt, 0, s, ev0, ev1, 0,
                                  segs, blk_seg, it);
        else
            hipExtLaunchKernelGGL(k_bicg_p<B, T, false, SOLO, PC, WIDE>, nb, nt, 0, s, ev0, ev1,
                                  0, segs, blk_seg, it);
    } else {
        hipExtLaunchKernelGGL(k_bicg_s<B, T, SOLO, PC, WIDE>, nb, nt, 0, s, ev0, ev1, 0, segs,
                              blk_seg, it, rec);
    }
}

// wide: the launch has more tiles than two resident workgroups per CU
// cover (FP32 with fracture blocks: the three-wave variant)
template <int B, typename T, bool SOLO, int PC>
static void part_impl(int which, const KSeg* segs, const int* blk_seg, int nblk_total, int it,
                      hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, SegStatus* rec, bool wide) {
    if (PC && wide && sizeof(T) == 4)
        part_impl_w<B, T, SOLO, PC, true>(which, segs, blk_seg, nblk_total, it, s, ev0, ev1, rec);
    else
        part_impl_w<B, T, SOLO, PC, false>(which, segs, blk_seg, nblk_total, it, s, ev0, ev1, rec);
}

int krylov_grid(int nA, int cap) { return std::min(kgrid(nA), std::max(1, cap)); }

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
        o.rr = S.kb.sc->rr;
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

void launch_ir_residual(int b, bool fp32, bool solo, const KSeg* segs, const int* blk_seg,
                        int nblk_total, bool x_zero, hipStream_t s) {
    if (nblk_total <= 0) return;
#define IR(BV, TT)                                                                         \
    do {                                                                                   \
        if (solo)                                                                          \
            k_ir_residual<BV, TT, true><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg,        \
                                                                     x_zero ? 1 : 0);      \
        else                                                                               \
            k_ir_residual<BV, TT, false><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg,       \
                                                                      x_zero ? 1 : 0);     \
    } while (0)
    KDISPATCH(IR)
#undef IR
}

void launch_bicg_part(int which, int b, bool fp32, bool solo, int pc, const KSeg* segs,
                      const int* blk_seg, int nblk_total, int it, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1, SegStatus* rec, bool wide) {
    if (nblk_total <= 0) return;
#define PJ(BV, TT, SO, PM) \
    part_impl<BV, TT, SO, PM>(which, segs, blk_seg, nblk_total, it, s, ev0, ev1, rec, wide)
#define PI(BV, TT)                                                                        \
    do {                                                                                  \
        if (solo) {                                                                       \
            if (pc == 2) PJ(BV, TT, true, 2);                                             \
            else if (pc) PJ(BV, TT, true, 1);                                             \
            else PJ(BV, TT, true, 0);                                                     \
        } else {                                                                          \
            if (pc == 2) PJ(BV, TT, false, 2);                                            \
            else if (pc) PJ(BV, TT, false, 1);                                            \
            else PJ(BV, TT, false, 0);                                                    \
        }                                                                                 \
    } while (0)
    KDISPATCH(PI)
#undef PI
#undef PJ
}

void launch_ir_accumulate(int b, bool fp32, bool solo, const KSeg* segs, const int* blk_seg,
                          int nblk_total, hipStream_t s) {
    if (nblk_total <= 0) return;
#define AC(BV, TT)                                                                          \
    do {                                                                                    \
        if (solo)                                                                           \
            k_ir_accumulate<BV, TT, true><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg);       \
        else                                                                                \
            k_ir_accumulate<BV, TT, false><<<nblk_total, KB_NT, 0, s>>>(segs, blk_seg);      \
    } while (0)
    KDISPATCH(AC)
#undef AC
}

} // namespace fimk
