// Fracture-block preconditioner for the local linear solve (Section 4.3
// leaves the solver open).  The hard part of these systems is the
// fracture network: fracture cells couple to each other through
// transmissibilities orders of magnitude above the matrix ones, while
// matrix rows are strongly diagonally dominant.  On top of the b x b
// block-Jacobi scaling (A~ = D^{-1} J), each run of consecutive local rows
// that belong to one fracture is grouped into a block of at most
// PC_DOF / b rows that never crosses a 256-row Krylov tile; the exact
// inverse of A~ restricted to the block is formed once per Newton
// iteration and applied on the left inside each Krylov product kernel
// (fim_krylov.hip).  Matrix rows and rows of one-row blocks keep the plain
// scaling.
#include "fim_device.hpp"

namespace fimk {

// Block layout of one local system, one workgroup per 256-row tile:
//   pcinfo[r] = (first row of r's block - tile base) << 16 | block rows
//   pcoff[r]  = element offset of the block's inverse in the inverse
//               store (grouped layout of fim_internal.hpp); the block's
//               first fracture cell ordinal times cell_stride, so the
//               blocks of one system never overlap.
__global__ __launch_bounds__(KB_NT) void k_pc_blocks(int nA, const int* __restrict__ l2g,
                                                     const int* __restrict__ frac_id,
                                                     const int* __restrict__ ford, int cap,
                                                     int cell_stride, int* __restrict__ pcinfo,
                                                     int* __restrict__ pcoff,
                                                     int* __restrict__ rows2) {
    __shared__ int sf[KB_NT];   // fracture id of each row (-1 matrix, -2 past nA)
    __shared__ int ss[KB_NT];   // block start of each row
    const int t = threadIdx.x, base = blockIdx.x * KB_NT, r = base + t;
    const bool valid = r < nA;
    const int f = valid ? frac_id[l2g[r]] : -2;
    sf[t] = f;
    __syncthreads();
    int run = t;
    if (f >= 0)
        while (run > 0 && sf[run - 1] == f) run--;
    const int bs = f >= 0 ? run + ((t - run) / cap) * cap : t;
    ss[t] = bs;
    __syncthreads();
    int size = 1;
    if (f >= 0) {
        int e = bs;
        while (e + 1 < KB_NT && ss[e + 1] == bs) e++;
        size = e - bs + 1;
    }
    if (valid) {
        pcinfo[r] = (bs << 16) | size;
        pcoff[r] = (size > 1) ? ford[l2g[base + bs]] * cell_stride : 0;
        if (size > 1 && bs == t) atomicAdd(rows2, size * size);   // sum of block rows^2
    }
}

void launch_pc_blocks(int nA, const int* l2g, const int* frac_id, const int* ford, int cap,
                      int cell_stride, int* pcinfo, int* pcoff, int* rows2, hipStream_t s) {
    launch_fill_i32(rows2, 1, 0, s);
    if (nA <= 0) return;
    k_pc_blocks<<<(nA + KB_NT - 1) / KB_NT, KB_NT, 0, s>>>(nA, l2g, frac_id, ford, cap,
                                                            cell_stride, pcinfo, pcoff, rows2);
}

// Inverse of every multi-row block of a tile, one wave per block, stored
// in FP32 (8-bit mantissas are not enough for nearly singular blocks): the
// block of A~ = D^{-1} J (the scaled blocks k_precond wrote, in the
// Krylov precision; FP32 from here on) is assembled
// in LDS, padded to 64 x 64 with the identity, and each lane takes one
// row into registers.  Gauss-Jordan elimination then runs 64 steps
// without pivoting (the scaled blocks have unit diagonal blocks and are
// diagonally dominant in practice); every step takes column 0 as the
// pivot column, broadcasts the pivot row through LDS, and shifts the
// columns left by one, appending the new column of the inverse at the end,
// so that all register indices are compile-time constants and after 64
// steps the registers hold the inverse in the original column order.  A
// pivot below 1e-20 in magnitude or a non-finite one, or an inverse entry
// above 1e8, leaves the identity for that block (plain block Jacobi on its
// rows).
constexpr int PCI_SUB = 8;    // single-wave workgroups per tile

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int B, typename T>
__global__ __launch_bounds__(WAVE) void k_pc_invert(int nA, LocalSys ls,
                                                    const T* __restrict__ At,
                                                    const int* __restrict__ pcinfo,
                                                    const int* __restrict__ pcoff,
                                                    float* __restrict__ pcM) {
    constexpr int BB = B * B;
    __shared__ __align__(16) float M[PC_DOF * PC_DOF];
    __shared__ int list[KB_NT];
    const int tile = blockIdx.x / PCI_SUB, sub = blockIdx.x % PCI_SUB;
    const int base = tile * KB_NT, lane = threadIdx.x;
    // the tile's multi-row blocks in row order (the same list in every
    // workgroup of the tile; workgroup sub takes blocks sub, sub + 8, ...)
    int nb = 0;
    for (int k = 0; k < KB_NT / WAVE; k++) {
        const int t = k * WAVE + lane, r = base + t;
        bool lead = false;
        if (r < nA) {
            const int info = pcinfo[r];
            lead = (info & 0xffff) > 1 && (info >> 16) == t;
        }
        const unsigned long long bal = __ballot(lead);
        if (lead) list[nb + __popcll(bal & ((1ull << lane) - 1ull))] = t;
        nb += __popcll(bal);
    }
    wave_sync();
    for (int q = sub; q < nb; q += PCI_SUB) {
        const int bs = list[q];
        const int size = pcinfo[base + bs] & 0xffff;
        const int N = size * B;
        for (int e = lane; e < N * N; e += WAVE) M[e] = 0.0f;
        wave_sync();
        if (lane < size) {
            // the row of A~: identity diagonal block, off-diagonal blocks
            // as scaled by k_precond (At, Krylov precision).  Columns of a
            // group of slots are loaded together, then their blocks.
            const int r = base + bs + lane;
            const long s0 = slot_of(ls, r, 0);
            const int width = ls.swidth[r / SLICE];
#pragma unroll
            for (int i = 0; i < B; i++) M[(lane * B + i) * N + lane * B + i] = 1.0f;
            for (int k0 = 1; k0 < width; k0 += 8) {
                int jl[8];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const int k = k0 + u;
                    jl[u] = k < width ? ls.col[s0 + (long)k * SLICE] - (base + bs) : -1;
                }
                T blk[8][BB];
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    const bool in = jl[u] >= 0 && jl[u] < size && jl[u] != lane;
#pragma unroll
                    for (int e = 0; e < BB; e++)
                        blk[u][e] = in ? At[(s0 + (long)min(k0 + u, width - 1) * SLICE) * BB + e]
                                       : (T)0;
                }
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if (!(jl[u] >= 0 && jl[u] < size && jl[u] != lane)) continue;
#pragma unroll
                    for (int i = 0; i < B; i++)
#pragma unroll
                        for (int j = 0; j < B; j++)
                            M[(lane * B + i) * N + jl[u] * B + j] = (float)blk[u][i * B + j];
                }
            }
        }
        wave_sync();
        float a[PC_DOF];
#pragma unroll
        for (int c = 0; c < PC_DOF; c++)
            a[c] = (lane < N && c < N) ? M[lane * N + c] : (c == lane ? 1.0f : 0.0f);
        wave_sync();
        bool bad = false;
        // N steps; afterwards columns 64 - N .. 63 of rows 0 .. N-1 hold the
        // inverse (the identity padding is never a pivot)
        for (int step = 0; step < N; step++) {
            if (lane == step) {
#pragma unroll
                for (int c = 0; c < PC_DOF; c++) M[c] = a[c];
            }
            wave_sync();
            float pr[PC_DOF];
#pragma unroll
            for (int c = 0; c < PC_DOF; c++) pr[c] = M[c];
            wave_sync();
            const float p = pr[0];
            bad = bad || !(fabsf(p) > 1e-20f) || !isfinite(p);
            const float ip = 1.0f / p;
            const float f = a[0];
            const bool me = lane == step;
#pragma unroll
            for (int c = 1; c < PC_DOF; c++) {
                const float sc = pr[c] * ip;
                a[c - 1] = me ? sc : a[c] - f * sc;
            }
            a[PC_DOF - 1] = me ? ip : -f * ip;
        }
        const int c0 = PC_DOF - N;
        bool big = false;
#pragma unroll
        for (int c = 0; c < PC_DOF; c++)
            if (lane < N && c >= c0 && !(fabsf(a[c]) <= 1e8f)) big = true;
        bad = bad || __any(big);
        // grouped store (see fim_internal.hpp): lane = unknown rr b + ci
        constexpr int K = pc_group_cols(B), W = B * K;
        float* out = pcM + pcoff[base + bs];
        const int rr = lane / B, ci = lane - rr * B;
        const int rowo = rr * W + ci * K, grp = size * W;
        if (lane < N) {
#pragma unroll
            for (int c = 0; c < PC_DOF; c++)
                if (c >= c0) {
                    const int j = c - c0;
                    out[(j / K) * grp + rowo + j % K] = bad ? (j == lane ? 1.0f : 0.0f) : a[c];
                }
            for (int j = N; j % K != 0; j++) out[(j / K) * grp + rowo + j % K] = 0.0f;
        }
        wave_sync();
    }
}

void launch_pc_invert(int b, bool fp32, int nA, const LocalSys& ls, const void* At,
                      const int* pcinfo, const int* pcoff, float* pcM, hipStream_t s) {
    if (nA <= 0) return;
    const int nb = (nA + KB_NT - 1) / KB_NT * PCI_SUB;
#define PV(BV, TT) \
    k_pc_invert<BV, TT><<<nb, WAVE, 0, s>>>(nA, ls, (const TT*)At, pcinfo, pcoff, pcM)
    if (fp32) {
        if (b == 1) PV(1, float); else if (b == 2) PV(2, float); else PV(3, float);
    } else {
        if (b == 1) PV(1, double); else if (b == 2) PV(2, double); else PV(3, double);
    }
#undef PV
}

} // namespace fimk
