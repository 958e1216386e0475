// Fracture-block preconditioner for the local linear solve (Section 4.3
// leaves the solver open).  The hard part of these systems is the
// fracture network: fracture cells couple to each other through
// transmissibilities orders of magnitude above the matrix ones, while
// matrix rows are strongly diagonally dominant.  On top of the b x b
// block-Jacobi scaling (A~ = D^{-1} J), each run of consecutive local rows
// that belong to one fracture is split into blocks of at most pc_cells(b)
// rows that never cross a 256-row Krylov tile; the exact
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
// and the list of multi-row blocks, (first row, rows) pairs in no
// particular order: cnt[1] entries; cnt[0] = sum of rows^2.
// A fracture's run of rows inside the tile covers units i0 .. iL of it
// (funit); it is cut into nb = ceil((iL - i0 + 1) / cap_units) blocks, block
// k taking the units from floor(k (iL - i0 + 1) / nb) on.  Whole units keep
// a layered fracture's pieces (the cells of one segment over its layers,
// coupled the most strongly) inside one block, and equal parts avoid a
// short leftover block.
// (vb: the tile)
__device__ inline void pc_blocks_tile(int nA, const int* __restrict__ l2g,
                                      const int* __restrict__ frac_id,
                                      const int* __restrict__ ford,
                                      const int* __restrict__ funit, int cell_stride,
                                      int* __restrict__ pcinfo, int* __restrict__ pcoff,
                                      int* __restrict__ list, int* __restrict__ cnt, int vb) {
    constexpr int NW = KB_NT / WAVE;
    __shared__ int sf[KB_NT];              // fracture id of each row (-1 matrix, -2 past nA)
    __shared__ int su[KB_NT];              // funit of each fracture row, then its block
    __shared__ int sfo[KB_NT];             // fracture-cell ordinal of each fracture row
    __shared__ int wfirst[NW], wlast[NW];  // first / last start in each wave
    __shared__ int nlead[NW], sq[NW + 1], base_q, wsq[NW];
    const int t = threadIdx.x, lane = t % WAVE, w = t / WAVE;
    const int base = vb * KB_NT, r = base + t;
    const bool valid = r < nA;
    const int cell = valid ? l2g[r] : 0;
    const int f = valid ? frac_id[cell] : -2;
    const int fu = f >= 0 ? funit[cell] : 0;
    sf[t] = f;
    su[t] = fu;
    sfo[t] = f >= 0 ? ford[cell] : 0;
    const unsigned long long upto = (2ull << lane) - 1ull;   // lanes 0 .. lane
    // the segment around row t of the rows flagged by st: from the last
    // flagged row at or before t to before the first one after it
    auto segment = [&](bool st, int& lo, int& hi) {
        const unsigned long long m = __ballot(st);
        if (lane == 0) {
            wfirst[w] = m ? w * WAVE + __ffsll((long long)m) - 1 : KB_NT;
            wlast[w] = m ? w * WAVE + 63 - __clzll((long long)m) : -1;
        }
        __syncthreads();
        lo = 0;
        hi = KB_NT;
        if (m & upto) {
            lo = w * WAVE + 63 - __clzll((long long)(m & upto));
        } else {
            for (int v = w - 1; v >= 0; v--)
                if (wlast[v] >= 0) { lo = wlast[v]; break; }
        }
        if (m & ~upto) {
            hi = w * WAVE + __ffsll((long long)(m & ~upto)) - 1;
        } else {
            for (int v = w + 1; v < NW; v++)
                if (wfirst[v] < KB_NT) { hi = wfirst[v]; break; }
        }
        __syncthreads();   // wfirst / wlast reused by the next call
    };
    __syncthreads();
    // runs of equal fracture id
    int run, rend;
    segment(t == 0 || sf[t - 1] != f, run, rend);
    // block k of the run's units (matrix rows and rows past nA: -1, one
    // row each)
    int k = -1;
    if (f >= 0) {
        const int i0 = su[run] >> 8, ru = (su[rend - 1] >> 8) - i0 + 1, cu = fu & 255;
        const int nb = (ru + cu - 1) / cu, iu = (fu >> 8) - i0;
        k = (int)(((long long)(iu + 1) * nb + ru - 1) / ru) - 1;
    }
    __syncthreads();   // su read above
    su[t] = k;
    __syncthreads();
    int bs, be;
    segment(t == 0 || f < 0 || sf[t - 1] != f || su[t - 1] != k, bs, be);
    const int size = be - bs;
    const bool lead = valid && size > 1 && bs == t;
    // list slots, and the sum of rows^2 over the blocks (profiling): one
    // atomic each per workgroup
    const unsigned long long lm = __ballot(lead);
    int s2 = lead ? size * size : 0;
    for (int o = WAVE / 2; o > 0; o /= 2) s2 += __shfl_xor(s2, o);
    if (lane == 0) {
        nlead[w] = __popcll(lm);
        wsq[w] = s2;
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0, a2 = 0;
        for (int v = 0; v < NW; v++) {
            sq[v] = acc;
            acc += nlead[v];
            a2 += wsq[v];
        }
        sq[NW] = acc;
        base_q = acc ? atomicAdd(&cnt[1], acc) : 0;
        if (a2) atomicAdd(&cnt[0], a2);
    }
    __syncthreads();
    if (valid) {
        pcinfo[r] = (bs << 16) | size;
        pcoff[r] = (size > 1) ? sfo[bs] * cell_stride : 0;
    }
    if (lead) {
        const int q = base_q + sq[w] + __popcll(lm & (upto >> 1));
        list[2 * q] = r;
        list[2 * q + 1] = size;
    }
}

__global__ __launch_bounds__(KB_NT) void k_pc_blocks(int nA, const int* __restrict__ l2g,
                                                     const int* __restrict__ frac_id,
                                                     const int* __restrict__ ford,
                                                     const int* __restrict__ funit,
                                                     int cell_stride, int* __restrict__ pcinfo,
                                                     int* __restrict__ pcoff,
                                                     int* __restrict__ list,
                                                     int* __restrict__ cnt) {
    pc_blocks_tile(nA, l2g, frac_id, ford, funit, cell_stride, pcinfo, pcoff, list, cnt,
                   blockIdx.x);
}

// batched: members with fracture blocks (their counters cleared before)
__global__ __launch_bounds__(KB_NT) void k_pc_blocks_seg(const BMember* __restrict__ t,
                                                         const BMap* __restrict__ map,
                                                         int cell_stride) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (!M.frac_id) return;
    pc_blocks_tile(M.nA, M.ls.l2g, M.frac_id, M.ford, M.funit, cell_stride, M.pcinfo, M.pcoff,
                   M.pclist, &M.dint[5], e.vb);
}

void launch_pc_blocks_seg(const BMember* t, const BMap* rows, int nrows, int cell_stride,
                          hipStream_t s) {
    if (nrows > 0) k_pc_blocks_seg<<<nrows, KB_NT, 0, s>>>(t, rows, cell_stride);
}

void launch_pc_blocks(int nA, const int* l2g, const int* frac_id, const int* ford,
                      const int* funit, int cell_stride, int* pcinfo, int* pcoff, int* list,
                      int* cnt, hipStream_t s) {
    launch_fill_i32(cnt, 2, 0, s);
    if (nA <= 0) return;
    k_pc_blocks<<<(nA + KB_NT - 1) / KB_NT, KB_NT, 0, s>>>(nA, l2g, frac_id, ford, funit,
                                                            cell_stride, pcinfo, pcoff, list, cnt);
}

// Inverse of every multi-row block of the list, one wave per block, stored
// in FP32 (8-bit mantissas are not enough for nearly singular blocks): the
// block of A~ = D^{-1} J (the scaled blocks k_precond wrote, in the
// Krylov precision; FP32 from here on) is assembled in LDS, padded to
// 64 x 64 with the identity, and each lane takes one row into registers.
// Gauss-Jordan elimination then runs N steps (N = the block's unknowns; the
// identity padding never pivots) without pivoting (the scaled blocks have
// unit diagonal blocks and are diagonally dominant in practice); every
// step takes column 0 as the pivot column, broadcasts the pivot row from
// the pivot lane's registers (lane reads, no LDS round trip), and shifts the
// columns left by one, appending the new column
// of the inverse at the end, so that all register indices are compile-time
// constants and after N steps columns 64 - N .. 63 hold the inverse.  Rows
// are eliminated with multiplier (entry / pivot) and the pivot row is left
// unscaled (one FMA per entry and step); each row is divided by its own
// pivot once at the end.  A
// pivot below 1e-20 in magnitude or a non-finite one, or an inverse entry
// above 1e8, leaves the identity for that block (plain block Jacobi on its
// rows).

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

typedef float f4v __attribute__((ext_vector_type(4)));

// the block in LDS, row stride MS (16-byte rows, offset banks per row)
constexpr int PCI_MS = PC_DOF + 4;

// Gauss-Jordan elimination of the block in M (rows 0 .. N-1 of the wave's
// lanes, C >= N register columns; the identity padding of M's rows is
// never a pivot): every step takes column 0 as the pivot column,
// broadcasts the pivot row from the pivot lane's registers (lane reads,
// no LDS round trip), eliminates with multiplier (entry / pivot), leaves
// the pivot row unscaled (one FMA per entry and step) and shifts the
// columns left by one, appending the new column of the inverse at the end,
// so all register indices are compile-time constants; each row is divided
// by its own pivot once at the end.  After N steps columns C - N .. C - 1
// hold the inverse; the rows go back to M.  Returns whether a pivot was
// below 1e-20 in magnitude or not finite.
template <int C, int MS = PCI_MS>
__device__ inline bool gauss_jordan(float* M, int N) {
    const int lane = threadIdx.x;
    float a[C];
    {
        const f4v* row = (const f4v*)&M[lane * MS];
#pragma unroll
        for (int c = 0; c < C / 4; c++) {
            const f4v v = row[c];
            a[4 * c] = v[0];
            a[4 * c + 1] = v[1];
            a[4 * c + 2] = v[2];
            a[4 * c + 3] = v[3];
        }
    }
    wave_sync();
    bool bad = false;
    float myip = 1.0f;   // 1 / this row's pivot
    for (int step = 0; step < N; step++) {
        float pr[C];
#pragma unroll
        for (int c = 0; c < C; c++)
            pr[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a[c]), step));
        const float p = pr[0];
        bad = bad || !(fabsf(p) > 1e-20f) || !isfinite(p);
        const float ip = 1.0f / p;
        const bool me = lane == step;
        if (me) myip = ip;
        const float f = me ? 0.0f : a[0] * ip;
#pragma unroll
        for (int c = 1; c < C; c++) a[c - 1] = fmaf(-f, pr[c], a[c]);
        a[C - 1] = me ? 1.0f : -f;
    }
#pragma unroll
    for (int c = 0; c < C; c++) a[c] *= myip;
    {
        f4v* row = (f4v*)&M[lane * MS];
#pragma unroll
        for (int c = 0; c < C / 4; c++)
            row[c] = f4v{a[4 * c], a[4 * c + 1], a[4 * c + 2], a[4 * c + 3]};
    }
    wave_sync();
    return bad;
}

// Gauss-Jordan elimination of G independent blocks of n rows at once (the
// decoupled blocks: one per unknown), block g in lanes g n .. g n + n - 1
// (n <= C, G n <= 64): the steps of gauss_jordan, with each lane taking
// the pivot row from its own block's pivot lane (a lane permute instead of
// a lane read, so one pass eliminates all G blocks).  Lanes from G n on
// hold no block (they pivot on themselves; nothing reads them).  Returns,
// per lane, whether a pivot of the lane's block was below 1e-20 in
// magnitude or not finite.
template <int C, int MS>
__device__ inline bool gauss_jordan_groups(float* M, int n, int G) {
    const int lane = threadIdx.x;
    const int grp = lane / n, r = lane - grp * n;
    const bool live = grp < G;
    float a[C];
    {
        const f4v* row = (const f4v*)&M[lane * MS];
#pragma unroll
        for (int c = 0; c < C / 4; c++) {
            const f4v v = row[c];
            a[4 * c] = v[0];
            a[4 * c + 1] = v[1];
            a[4 * c + 2] = v[2];
            a[4 * c + 3] = v[3];
        }
    }
    wave_sync();
    bool bad = false;
    float myip = 1.0f;
    const int base = (live ? grp * n : lane) * 4;   // byte address of lane grp n
    for (int step = 0; step < n; step++) {
        const int src = base + (live ? step * 4 : 0);
        float pr[C];
#pragma unroll
        for (int c = 0; c < C; c++)
            pr[c] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(a[c])));
        const float p = pr[0];
        bad = bad || !(fabsf(p) > 1e-20f) || !isfinite(p);
        const float ip = 1.0f / p;
        const bool me = !live || r == step;
        if (me) myip = ip;
        const float f = me ? 0.0f : a[0] * ip;
#pragma unroll
        for (int c = 1; c < C; c++) a[c - 1] = fmaf(-f, pr[c], a[c]);
        a[C - 1] = me ? 1.0f : -f;
    }
#pragma unroll
    for (int c = 0; c < C; c++) a[c] *= myip;
    {
        f4v* row = (f4v*)&M[lane * MS];
#pragma unroll
        for (int c = 0; c < C / 4; c++)
            row[c] = f4v{a[4 * c], a[4 * c + 1], a[4 * c + 2], a[4 * c + 3]};
    }
    wave_sync();
    return live && bad;
}

// register columns of a decoupled block (at most pc_cells(b) cells) and
// its LDS row stride
constexpr int PCI_DEC_C = 24;
constexpr int PCI_DEC_MS = PCI_DEC_C + 4;
static_assert(pc_cells(2) <= PCI_DEC_C && pc_cells(3) <= PCI_DEC_C,
              "decoupled blocks exceed their register columns");

// Block q of one system's list, by one wave; M: PC_DOF x PCI_MS floats of
// LDS.  Coupled: one inversion of A~ over all the block's unknowns (rows
// b x rows b, unknown-interleaved).  Decoupled (b > 1): A~ restricted to
// each unknown over the block's cells, the b blocks side by side in the
// lanes (unknown c's rows at lanes c rows ..) and eliminated together.
// Loops stay rolled where they run once per block: each wave runs this
// code about once per launch, so its size (instruction fetch) costs more
// than loop overhead.
template <int B, typename T, bool DEC>
__device__ void invert_block(const LocalSys& ls, const T* __restrict__ At,
                             const int* __restrict__ list, const int* __restrict__ pcoff,
                             float* __restrict__ pcM, int q, float* M) {
    constexpr int BB = B * B;
    constexpr bool dec = DEC && B > 1;
    constexpr int MS = dec ? PCI_DEC_MS : PCI_MS;
    const int lane = threadIdx.x;
    const int r0 = list[2 * q], size = list[2 * q + 1];
    // slot widths of the (at most two) slices the block's rows are in
    const int sl0 = r0 / SLICE, sl1 = (r0 + size - 1) / SLICE;
    const int w0 = ls.swidth[sl0], w1 = ls.swidth[sl1];
    const int N = dec ? size : size * B;   // rows of each inversion
    // the register width: the fewest of 32, 48 or 64 columns that hold
    // the block (columns C - N .. C - 1 end up holding the inverse)
    const int C = dec ? PCI_DEC_C : N <= 32 ? 32 : N <= 48 ? 48 : PC_DOF;
    // identity: the diagonal blocks of A~ and the padding
    {
        f4v* row = (f4v*)&M[lane * MS];
#pragma unroll 1
        for (int c = 0; c < C / 4; c++) {
            f4v z = {0.0f, 0.0f, 0.0f, 0.0f};
            const int d = dec ? lane % size : lane;   // the row's own column
            if (c == d / 4) z[d % 4] = 1.0f;
            row[c] = z;
        }
    }
    wave_sync();
    // off-diagonal blocks inside the block, from the scaled blocks
    // k_precond wrote (At, Krylov precision): the (slot, row) pairs of the
    // block are spread over the lanes, FU per lane at a time, the column
    // loads first, then the blocks that couple two rows
    constexpr int FU = 4;
    const int items = size * (max(w0, w1) - 1);
#pragma unroll 1
    for (int i0 = 0; i0 < items; i0 += WAVE * FU) {
        int jl[FU], rl[FU];
        long ps[FU];
#pragma unroll
        for (int u = 0; u < FU; u++) {
            const int i = i0 + u * WAVE + lane;
            const int k = 1 + i / size, rr = i - (k - 1) * size, r = r0 + rr;
            const bool ok = i < items && k < ((r / SLICE == sl0) ? w0 : w1);
            rl[u] = rr;
            ps[u] = ok ? slot_of(ls, r, k) : 0;
            jl[u] = ok ? ls.col[ps[u]] - r0 : -1;
        }
        T blk[FU][BB];
#pragma unroll
        for (int u = 0; u < FU; u++) {
            const bool in = jl[u] >= 0 && jl[u] < size && jl[u] != rl[u];
#pragma unroll
            for (int e = 0; e < BB; e++)   // decoupled: the diagonal entries only
                blk[u][e] = in && (!dec || e % (B + 1) == 0) ? At[ps[u] * BB + e] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < FU; u++) {
            if (!(jl[u] >= 0 && jl[u] < size && jl[u] != rl[u])) continue;
#pragma unroll
            for (int i = 0; i < B; i++)
#pragma unroll
                for (int j = 0; j < B; j++)
                    if (!dec)
                        M[(rl[u] * B + i) * MS + jl[u] * B + j] = (float)blk[u][i * B + j];
                    else if (i == j)   // unknown i of both cells: block i
                        M[(i * size + rl[u]) * MS + jl[u]] = (float)blk[u][i * B + j];
        }
    }
    wave_sync();
    bool bad;
    if constexpr (dec) {
        bad = gauss_jordan_groups<PCI_DEC_C, MS>(M, size, B);
    } else {
        if (N <= 32)
            bad = gauss_jordan<32>(M, N);
        else if (N <= 48)
            bad = gauss_jordan<48>(M, N);
        else
            bad = gauss_jordan<PC_DOF>(M, N);
    }
    const int c0 = C - N, nrow = dec ? B * size : N;
    if (lane < nrow) {
#pragma unroll 1
        for (int j = 0; j < N; j++) bad = bad || !(fabsf(M[lane * MS + c0 + j]) <= 1e8f);
    }
    // a failed inversion leaves the identity: the whole block (coupled) or
    // the unknown's block (decoupled)
    const unsigned long long bm = __ballot(bad);
    const int gi = dec ? lane / size : 0, gn = dec ? size : N;
    const unsigned long long gm = gn >= 64 ? ~0ull : ((1ull << gn) - 1) << (gi * gn);
    bad = (bm & gm) != 0;
    constexpr int K = pc_group_cols(B), W = B * K;
    typedef float kv __attribute__((ext_vector_type(K)));
    float* out = pcM + pcoff[r0];
    // lane: unknown rr b + ci of the block (coupled; the layout's columns
    // are the block's unknowns), or cell rr, unknown ci (decoupled; the
    // layout's columns are the block's cells)
    const int rr = dec ? lane - gi * size : lane / B, ci = dec ? gi : lane - rr * B;
    const int rowo = rr * W + ci * K, grp = size * W;
    const int diag = dec ? rr : lane;   // the row's own column (identity)
    if (lane < nrow) {
#pragma unroll 1
        for (int g = 0; g * K < N; g++) {
            kv v;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int j = g * K + k;
                v[k] = j >= N ? 0.0f : bad ? (j == diag ? 1.0f : 0.0f) : M[lane * MS + c0 + j];
            }
            *(kv*)(out + g * grp + rowo) = v;
        }
    }
    wave_sync();
}

// One system: workgroup w takes blocks w, w + grid, ... of its list.
// (DEC: decoupled blocks, whose 24-column rows need less LDS, so that more
// workgroups fit on a CU)
template <int B, typename T, bool DEC>
__global__ __launch_bounds__(WAVE) void k_pc_invert(LocalSys ls, const T* __restrict__ At,
                                                    const int* __restrict__ list,
                                                    const int* __restrict__ cnt,
                                                    const int* __restrict__ pcoff,
                                                    float* __restrict__ pcM) {
    __shared__ __align__(16) float M[PC_DOF * (DEC && B > 1 ? PCI_DEC_MS : PCI_MS)];
    const int nblk = *cnt;
    for (int q = blockIdx.x; q < nblk; q += gridDim.x)
        invert_block<B, T, DEC>(ls, At, list, pcoff, pcM, q, M);
}

// Many systems (a batch): the blocks of all lists in one sequence; pref
// holds the running block counts (pref[k] = blocks of systems 0 .. k-1).
__global__ __launch_bounds__(64) void k_pc_prefix(const PcSeg* __restrict__ segs, int nseg,
                                                  int* __restrict__ pref) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < nseg; k++) {
            pref[k] = acc;
            acc += *segs[k].cnt;
        }
        pref[nseg] = acc;
    }
}

template <int B, typename T, bool DEC>
__global__ __launch_bounds__(WAVE) void k_pc_invert_batch(const PcSeg* __restrict__ segs,
                                                          int nseg,
                                                          const int* __restrict__ pref) {
    __shared__ __align__(16) float M[PC_DOF * (DEC && B > 1 ? PCI_DEC_MS : PCI_MS)];
    const int total = pref[nseg];
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        int lo = 0, hi = nseg - 1;   // the system k with pref[k] <= q < pref[k + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (pref[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const PcSeg& S = segs[lo];
        invert_block<B, T, DEC>(S.ls, (const T*)S.At, S.list, S.pcoff, S.pcM, q - pref[lo], M);
    }
}

void launch_pc_invert(int b, bool fp32, int grid, const LocalSys& ls, const void* At,
                      const int* list, const int* cnt, const int* pcoff, float* pcM,
                      bool dec, hipStream_t s) {
    if (grid <= 0) return;
#define PV(BV, TT)                                                                    \
    do {                                                                              \
        if (dec)                                                                      \
            k_pc_invert<BV, TT, true><<<grid, WAVE, 0, s>>>(ls, (const TT*)At, list, cnt, \
                                                            pcoff, pcM);              \
        else                                                                          \
            k_pc_invert<BV, TT, false><<<grid, WAVE, 0, s>>>(ls, (const TT*)At, list,   \
                                                             cnt, pcoff, pcM);        \
    } while (0)
    if (fp32) {
        if (b == 1) PV(1, float); else if (b == 2) PV(2, float); else PV(3, float);
    } else {
        if (b == 1) PV(1, double); else if (b == 2) PV(2, double); else PV(3, double);
    }
#undef PV
}

void launch_pc_invert_batch(int b, bool fp32, int grid, const PcSeg* segs, int nseg, int* pref,
                            bool dec, hipStream_t s) {
    if (grid <= 0 || nseg <= 0) return;
    k_pc_prefix<<<1, 64, 0, s>>>(segs, nseg, pref);
#define PV(BV, TT)                                                              \
    do {                                                                        \
        if (dec) k_pc_invert_batch<BV, TT, true><<<grid, WAVE, 0, s>>>(segs, nseg, pref);  \
        else k_pc_invert_batch<BV, TT, false><<<grid, WAVE, 0, s>>>(segs, nseg, pref);     \
    } while (0)
    if (fp32) {
        if (b == 1) PV(1, float); else if (b == 2) PV(2, float); else PV(3, float);
    } else {
        if (b == 1) PV(1, double); else if (b == 2) PV(2, double); else PV(3, double);
    }
#undef PV
}

} // namespace fimk
