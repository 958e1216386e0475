// Active-set estimation (Algorithms 1 and 2), compaction of the active
// rows (the restriction R_A of Section 4.3) and the sliced-ELL structure of
// the local system.
//
// * compaction: one 4096-cell tile per block; each thread owns 16 flags,
//   a wave ballot counts the active ones and a block scan orders them, so
//   l2g comes out ascending and g2l is the inverse map (-1 = inactive);
//   tile offsets are prefix sums of the per-tile counts (two launches, no
//   spin waits, deterministic);
// * neighbourhood marking: level by level from the seed cells (the
//   boundary cells with a non-negligible update), one launch per layer over
//   a byte array of graph distances; a cell reached in pass k gets the
//   value k whichever thread writes it, so the set is the same in any
//   schedule;
// * the slice width of the sliced-ELL matrix is the wave maximum of the
//   active-neighbour counts of its 64 rows;
// * the residual-based set: the cells whose residual error measure reaches
//   the tolerance, inflated by the same level-by-level marking.
#include "fim_device.hpp"

namespace fimk {

__global__ void k_fill_u8(uint8_t* a, int n, uint8_t v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}
__global__ void k_fill_i32(int* a, int n, int v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}
__global__ void k_fill_f64(double* a, long n, double v) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// lane w copies word w (vector stores into the mapped host buffers)
__global__ __launch_bounds__(64) void k_status_out(const NStat* __restrict__ ns,
                                                   const int* __restrict__ dint,
                                                   NStat* __restrict__ ons, int* __restrict__ oint) {
    constexpr int NW = (int)(sizeof(NStat) / sizeof(int));
    static_assert(sizeof(NStat) % sizeof(int) == 0 && NW <= 60, "NStat words");
    const int w = threadIdx.x;
    if (ns && w < NW) ((int*)ons)[w] = ((const int*)ns)[w];
    if (w >= 60) oint[w - 60] = dint[w - 60];
}

void launch_status_out(const NStat* ns, const int* dint, NStat* ons, int* oint, hipStream_t s) {
    k_status_out<<<1, 64, 0, s>>>(ns, dint, ons, oint);
}

void launch_fill_u8(uint8_t* a, int n, uint8_t v, hipStream_t s) {
    if (n > 0) k_fill_u8<<<nblocks(n), NT, 0, s>>>(a, n, v);
}
void launch_fill_i32(int* a, int n, int v, hipStream_t s) {
    if (n > 0) k_fill_i32<<<nblocks(n), NT, 0, s>>>(a, n, v);
}
void launch_fill_f64(double* a, long n, double v, hipStream_t s) {
    if (n > 0) k_fill_f64<<<nblocks(n), NT, 0, s>>>(a, n, v);
}

// ------------------------------------------------------------ compaction
constexpr int PER = TILE / NT;   // 16 cells per thread

// (vb: the tile; the bodies below take the workgroup's index within its
// own system, so that the batched launches share them).  Cell q NT + t of
// a tile belongs to thread t (round q), so every load and store of a round
// is one contiguous span per wave.
__device__ inline void compact_count(const uint8_t* __restrict__ act, int n,
                                     int* __restrict__ blk_cnt, int vb) {
    const int base = vb * TILE + threadIdx.x;
    int c = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = base + q * NT;
        if (i < n && act[i]) c++;
    }
    c = block_sum_i(c);
    if (threadIdx.x == 0) blk_cnt[vb] = c;
}

__global__ __launch_bounds__(NT) void k_compact_count(const uint8_t* __restrict__ act, int n,
                                                      int* __restrict__ blk_cnt) {
    compact_count(act, n, blk_cnt, blockIdx.x);
}

// (vb of ntile tiles; the last one writes n_out).  The tile's cells in
// index order are rounds q, then waves w, then lanes: each wave takes the
// mask of its active cells per round (ballot), the PER x NW counts are
// scanned in that order in LDS, and a cell's position is its tile's
// offset + its (round, wave) offset + the active lanes below it.
__device__ inline void compact_scatter(const uint8_t* __restrict__ act, int n,
                                       const int* __restrict__ blk_cnt, int* __restrict__ l2g,
                                       int* __restrict__ g2l, int* __restrict__ n_out, int vb,
                                       int ntile) {
    constexpr int NW = NT / WAVE;
    static_assert(PER * NW <= WAVE, "one wave scans the round counts");
    __shared__ int cnt[PER * NW];
    // offset of this tile: sum of the preceding tile counts
    int off = 0;
    for (int t = threadIdx.x; t < vb; t += NT) off += blk_cnt[t];
    off = block_sum_i(off);
    const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
    const int base = vb * TILE + threadIdx.x;
    unsigned long long mask[PER];
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = base + q * NT;
        mask[q] = __ballot(i < n && act[i]);
        if (lane == 0) cnt[q * NW + w] = __popcll(mask[q]);
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {   // exclusive scan of the PER x NW counts
        const int v = threadIdx.x < PER * NW ? cnt[threadIdx.x] : 0;
        int inc = v;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const int y = __shfl_up(inc, o, WAVE);
            if (lane >= o) inc += y;
        }
        if (threadIdx.x < PER * NW) cnt[threadIdx.x] = inc - v;
        if (vb == ntile - 1 && threadIdx.x == WAVE - 1) *n_out = off + inc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int i = base + q * NT;
        if (i >= n) break;
        const unsigned long long m = mask[q];
        if ((m >> lane) & 1ull) {
            const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
            const int pos = off + cnt[q * NW + w] + below;
            l2g[pos] = i;
            g2l[i] = pos;
        } else {
            g2l[i] = -1;
        }
    }
}

__global__ __launch_bounds__(NT) void k_compact_scatter(const uint8_t* __restrict__ act, int n,
                                                        const int* __restrict__ blk_cnt,
                                                        int* __restrict__ l2g,
                                                        int* __restrict__ g2l,
                                                        int* __restrict__ n_out) {
    compact_scatter(act, n, blk_cnt, l2g, g2l, n_out, blockIdx.x, gridDim.x);
}

// batched: the FIM_LOCAL and FIM_RESID members (tile launches)
__global__ __launch_bounds__(NT) void k_compact_count_seg(const BMember* __restrict__ t,
                                                          const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (!M.compact) return;
    compact_count(M.act, M.n, M.blk, e.vb);
}

__global__ __launch_bounds__(NT) void k_compact_scatter_seg(const BMember* __restrict__ t,
                                                            const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (!M.compact) return;
    compact_scatter(M.act, M.n, M.blk, (int*)M.ls.l2g, (int*)M.ls.g2l, &M.dint[1], e.vb,
                    (M.n + TILE - 1) / TILE);
}

void launch_compact_seg(const BMember* t, const BMap* tiles, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    k_compact_count_seg<<<ntiles, NT, 0, s>>>(t, tiles);
    k_compact_scatter_seg<<<ntiles, NT, 0, s>>>(t, tiles);
}

void launch_compact(const uint8_t* act, int n, int* blk_cnt, int* l2g,
                    int* g2l, int* n_out, hipStream_t s) {
    const int nt = (n + TILE - 1) / TILE;
    k_compact_count<<<nt, NT, 0, s>>>(act, n, blk_cnt);
    k_compact_scatter<<<nt, NT, 0, s>>>(act, n, blk_cnt, l2g, g2l, n_out);
}

// ------------------------------------------------------------- structure
__device__ inline void slice_width(int nA, const int* __restrict__ l2g,
                                   const int* __restrict__ g2l, const Graph& g,
                                   int* __restrict__ swidth, int* __restrict__ nnzb, int vb) {
    const int r = vb * NT + threadIdx.x;
    int cnt = 0;
    if (r < nA) {
        const int i = l2g[r];
        cnt = 1;
        for (int e = g.adj_ptr[i]; e < g.adj_ptr[i + 1]; e++)
            cnt += (g2l[g.adj_nbr[e]] >= 0) ? 1 : 0;
    }
    const int tot = block_sum_i(cnt);
    if (threadIdx.x == 0 && tot) atomicAdd(nnzb, tot);
    cnt = wave_max_i(cnt);
    if ((threadIdx.x % WAVE) == 0 && r < nA) swidth[r / SLICE] = cnt;
}

__global__ __launch_bounds__(NT) void k_slice_width(int nA, const int* __restrict__ l2g,
                                                    const int* __restrict__ g2l, Graph g,
                                                    int* __restrict__ swidth,
                                                    int* __restrict__ nnzb) {
    slice_width(nA, l2g, g2l, g, swidth, nnzb, blockIdx.x);
}

void launch_structure(int nA, const int* l2g, const int* g2l, const Graph& g,
                      int* swidth, int* nnzb, hipStream_t s) {
    launch_fill_i32(nnzb, 1, 0, s);
    if (nA <= 0) return;
    k_slice_width<<<nblocks(nA), NT, 0, s>>>(nA, l2g, g2l, g, swidth, nnzb);
}

// -------------------------------------------------------------- boundary
// V_B: active cells with at least one inactive neighbour.
__device__ inline void boundary_rows(int nA, const int* __restrict__ l2g,
                                     const int* __restrict__ g2l, const Graph& g,
                                     uint8_t* __restrict__ bnd, int* __restrict__ count,
                                     int vb) {
    const int r = vb * NT + threadIdx.x;
    int b = 0;
    if (r < nA) {
        const int i = l2g[r];
        for (int e = g.adj_ptr[i]; e < g.adj_ptr[i + 1]; e++)
            if (g2l[g.adj_nbr[e]] < 0) { b = 1; break; }
        bnd[i] = (uint8_t)b;
    }
    b = block_sum_i(b);
    if (threadIdx.x == 0 && b) atomicAdd(count, b);
}

__global__ __launch_bounds__(NT) void k_boundary(int nA, const int* __restrict__ l2g,
                                                 const int* __restrict__ g2l, Graph g,
                                                 uint8_t* __restrict__ bnd,
                                                 int* __restrict__ count) {
    boundary_rows(nA, l2g, g2l, g, bnd, count, blockIdx.x);
}

void launch_boundary(int nA, const int* l2g, const int* g2l, const Graph& g,
                     uint8_t* bnd, int* count, hipStream_t s) {
    if (nA > 0) k_boundary<<<nblocks(nA), NT, 0, s>>>(nA, l2g, g2l, g, bnd, count);
}

// ------------------------------------------------- neighbourhood marking
// V_nbr^{i,m} of a set of seed cells: every cell within graph distance m
// of a seed.  Level-synchronous: lvl[n] holds the distance found so far
// (0xff: none); pass k marks the unmarked neighbours of the cells at
// distance k - 1.  A cell can be written by several threads in one pass,
// always with the same value k, and a cell at distance k - 1 is never
// rewritten in pass k, so the result is the same in any order.
__device__ inline void ball_step(int n, const Graph& g, int k, uint8_t* __restrict__ lvl,
                                 uint8_t* act, uint8_t* act2, int vb) {
    const int i = vb * NT + threadIdx.x;
    if (i >= n || lvl[i] != k - 1) return;
    const int e = g.adj_ptr[i + 1];
    for (int p = g.adj_ptr[i]; p < e; p++) {
        const int j = g.adj_nbr[p];
        if (lvl[j] > k) {
            lvl[j] = (uint8_t)k;
            act[j] = 1;
            if (act2) act2[j] = 1;
        }
    }
}

__global__ __launch_bounds__(NT) void k_ball_step(int n, Graph g, int k,
                                                  uint8_t* __restrict__ lvl, uint8_t* act,
                                                  uint8_t* act2) {
    ball_step(n, g, k, lvl, act, act2, blockIdx.x);
}

static void ball_steps(int n, const Graph& g, int m, uint8_t* lvl, uint8_t* act, uint8_t* act2,
                       hipStream_t s) {
    for (int k = 1; k <= m; k++)
        k_ball_step<<<nblocks(n), NT, 0, s>>>(n, g, k, lvl, act, act2);
}

// Algorithm 1/2 expansion seeds: i in V_B with |dp_i| >= eps (level 0,
// marked in V_A and the optional second set); *flag = 1 if any
__device__ inline void expand_seeds(int nA, const int* __restrict__ l2g,
                                    const uint8_t* __restrict__ bnd,
                                    const double* __restrict__ dp_abs, double eps,
                                    uint8_t* __restrict__ lvl, uint8_t* act, uint8_t* act2,
                                    int* flag, int vb) {
    const int r = vb * NT + threadIdx.x;
    int hit = 0;
    if (r < nA) {
        const int i = l2g[r];
        if (bnd[i] && dp_abs[i] >= eps) {
            hit = 1;
            lvl[i] = 0;
            act[i] = 1;
            if (act2) act2[i] = 1;
        }
    }
    hit = block_sum_i(hit);
    if (threadIdx.x == 0 && hit) atomicOr(flag, 1);
}

__global__ __launch_bounds__(NT) void k_expand_seeds(int nA, const int* __restrict__ l2g,
                                                     const uint8_t* __restrict__ bnd,
                                                     const double* __restrict__ dp_abs,
                                                     double eps, uint8_t* __restrict__ lvl,
                                                     uint8_t* act, uint8_t* act2, int* flag) {
    expand_seeds(nA, l2g, bnd, dp_abs, eps, lvl, act, act2, flag, blockIdx.x);
}

void launch_mark_expand(int nA, const int* l2g, const uint8_t* bnd,
                        const double* dp_abs, double eps, int m,
                        const Graph& g, uint8_t* act, uint8_t* act2,
                        int* flag, uint8_t* lvl, hipStream_t s) {
    if (nA <= 0) return;
    launch_fill_u8(lvl, g.n, 0xff, s);
    k_expand_seeds<<<nblocks(nA), NT, 0, s>>>(nA, l2g, bnd, dp_abs, eps, lvl, act, act2, flag);
    ball_steps(g.n, g, m < MAX_LAYERS ? m : MAX_LAYERS, lvl, act, act2, s);
}

// Residual-based set (the estimator of Lu and Beckner, Sections 1 and 4.2):
// the cells with err_i >= tol (level 0, *count = their number) and every
// cell within m layers of them; act is rewritten on all n cells.
__device__ inline void resid_seeds(int n, const double* __restrict__ err, double tol,
                                   uint8_t* __restrict__ lvl, uint8_t* __restrict__ act,
                                   int* count, int vb) {
    const int i = vb * NT + threadIdx.x;
    int hit = 0;
    if (i < n) {
        hit = err[i] >= tol ? 1 : 0;
        lvl[i] = hit ? 0 : 0xff;
        act[i] = (uint8_t)hit;
    }
    hit = block_sum_i(hit);
    if (threadIdx.x == 0 && hit) atomicAdd(count, hit);
}

__global__ __launch_bounds__(NT) void k_resid_seeds(int n, const double* __restrict__ err,
                                                    double tol, uint8_t* __restrict__ lvl,
                                                    uint8_t* __restrict__ act, int* count) {
    resid_seeds(n, err, tol, lvl, act, count, blockIdx.x);
}

void launch_mark_resid(int n, const double* err, double tol, int m, const Graph& g,
                       uint8_t* act, int* count, uint8_t* lvl, hipStream_t s) {
    if (n <= 0) return;
    k_resid_seeds<<<nblocks(n), NT, 0, s>>>(n, err, tol, lvl, act, count);
    ball_steps(n, g, m < MAX_LAYERS ? m : MAX_LAYERS, lvl, act, nullptr, s);
}

// Algorithm 1 shrink (only when no boundary update was non-negligible):
// V_A = supp du_A plus the always-active cells.
__device__ inline void shrink_rows(int nA, const int* __restrict__ l2g,
                                   const double* __restrict__ dp_abs, double eps, const Graph& g,
                                   uint8_t* act, const int* flag, int vb) {
    if (*flag) return;
    const int r = vb * NT + threadIdx.x;
    if (r >= nA) return;
    const int i = l2g[r];
    act[i] = (dp_abs[i] >= eps || (g.flags[i] & CF_AA)) ? 1 : 0;
}

__global__ __launch_bounds__(NT) void k_shrink(int nA, const int* __restrict__ l2g,
                                               const double* __restrict__ dp_abs, double eps,
                                               Graph g, uint8_t* act, const int* flag) {
    shrink_rows(nA, l2g, dp_abs, eps, g, act, flag, blockIdx.x);
}

// ---------------------------------------------- batched set launches
// Algorithm 1 after the update (FIM_LOCAL members): the expansion seeds
// (boundary cells with |dp| >= eps_loc) and their layers-layer
// neighbourhood, else the shrink; the residual-based marking (FIM_RESID
// members, error measure already in last_dp); FIM_FULL members: nothing.
// Same kernels and order as a member alone.
__global__ __launch_bounds__(NT) void k_sets_init_seg(const BMember* __restrict__ t,
                                                      const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode == FIM_LOCAL) {
        const int i = e.vb * NT + threadIdx.x;
        if (i < M.n) M.lvl[i] = 0xff;
    } else if (M.mode == FIM_RESID) {
        resid_seeds(M.n, M.last_dp, M.eps_res, M.lvl, M.act, M.dint, e.vb);
    }
}

__global__ __launch_bounds__(NT) void k_expand_seeds_seg(const BMember* __restrict__ t,
                                                         const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode != FIM_LOCAL) return;
    expand_seeds(M.nA, M.ls.l2g, M.bnd, M.dp_abs, M.eps_loc, M.lvl, M.act, nullptr, M.dint,
                 e.vb);
}

__global__ __launch_bounds__(NT) void k_ball_step_seg(const BMember* __restrict__ t,
                                                      const BMap* __restrict__ map, int k) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode == FIM_FULL || k > M.layers) return;
    ball_step(M.n, M.g, k, M.lvl, M.act, nullptr, e.vb);
}

__global__ __launch_bounds__(NT) void k_shrink_seg(const BMember* __restrict__ t,
                                                   const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode != FIM_LOCAL) return;
    shrink_rows(M.nA, M.ls.l2g, M.dp_abs, M.eps_loc, M.g, M.act, M.dint, e.vb);
}

void launch_ball_steps_seg(const BMember* t, const BMap* cells, int ncells, int layers,
                           hipStream_t s) {
    for (int k = 1; k <= (layers < MAX_LAYERS ? layers : MAX_LAYERS); k++)
        k_ball_step_seg<<<ncells, NT, 0, s>>>(t, cells, k);
}

__global__ __launch_bounds__(NT) void k_support_seg(const BMember* __restrict__ t,
                                                    const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (!M.commit) return;
    const int i = e.vb * NT + threadIdx.x;
    if (i >= M.n) return;
    M.supp[i] = (fabs(M.u[i] - M.un[i]) >= M.eps_loc || (M.g.flags[i] & CF_AA)) ? 1 : 0;
}

void launch_support_seg(const BMember* t, const BMap* cells, int ncells, hipStream_t s) {
    if (ncells > 0) k_support_seg<<<ncells, NT, 0, s>>>(t, cells);
}

void launch_sets_seg(int fk, const BMember* t, const BMap* rows, int nrows, const BMap* cells,
                     int ncells, const BMap* mem, int nmem, int layers, bool any_resid,
                     hipStream_t s) {
    (void)mem;
    (void)nmem;
    if (ncells <= 0) return;
    if (any_resid) launch_resid_err_seg(fk, t, cells, ncells, s);
    k_sets_init_seg<<<ncells, NT, 0, s>>>(t, cells);
    if (nrows > 0) k_expand_seeds_seg<<<nrows, NT, 0, s>>>(t, rows);
    launch_ball_steps_seg(t, cells, ncells, layers, s);
    if (nrows > 0) k_shrink_seg<<<nrows, NT, 0, s>>>(t, rows);
}

// Workgroup maps of the batched launches from the members' workgroup
// counts: pref holds three exclusive prefix arrays of K + 1 ints (row,
// cell and tile workgroups); map k gets, for each workgroup b < pref_k[K],
// the member q with pref_k[q] <= b < pref_k[q + 1] and b - pref_k[q]; mem
// lists the members.
__global__ __launch_bounds__(NT) void k_build_maps(const int* __restrict__ pref, int K,
                                                   BMap* __restrict__ rows,
                                                   BMap* __restrict__ cells,
                                                   BMap* __restrict__ tiles,
                                                   BMap* __restrict__ mem) {
    const int b = blockIdx.x * NT + threadIdx.x;
    BMap* const out[3] = {rows, cells, tiles};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const int* p = pref + k * (K + 1);
        if (b < p[K]) {
            int lo = 0, hi = K - 1;   // last q with p[q] <= b
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (p[mid] <= b) lo = mid;
                else hi = mid - 1;
            }
            out[k][b] = BMap{lo, b - p[lo]};
        }
    }
    if (b < K) mem[b] = BMap{b, 0};
}

void launch_build_maps(const int* pref, int K, int most, BMap* rows, BMap* cells, BMap* tiles,
                       BMap* mem, hipStream_t s) {
    const int w = most > K ? most : K;
    if (w > 0) k_build_maps<<<nblocks(w), NT, 0, s>>>(pref, K, rows, cells, tiles, mem);
}

// status words of every member (one workgroup of 64 per member)
__global__ void k_status_seg(const BMember* __restrict__ t, const BMap* __restrict__ map,
                             BStatus* out) {
    const int q = map[blockIdx.x].q;
    const BMember& M = t[q];
    if (threadIdx.x == 0) {
        out[q].ns = *M.ns;
#pragma unroll
        for (int k = 0; k < 4; k++) out[q].dint[k] = M.dint[k];
    }
}

void launch_status_seg(const BMember* t, const BMap* mem, int nmem, BStatus* out,
                       hipStream_t s) {
    if (nmem > 0) k_status_seg<<<nmem, 64, 0, s>>>(t, mem, out);
}

// the counters of the structure pass: matrix blocks, fracture blocks,
// boundary size
__global__ void k_struct_reset_seg(const BMember* __restrict__ t, const BMap* __restrict__ map) {
    const BMember& M = t[map[blockIdx.x].q];
    if (threadIdx.x == 0) {
        M.dint[2] = 0;
        M.dint[4] = 0;
        M.dint[5] = 0;
        M.dint[6] = 0;
    }
}

__global__ __launch_bounds__(NT) void k_slice_width_seg(const BMember* __restrict__ t,
                                                        const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    slice_width(M.nA, M.ls.l2g, M.ls.g2l, M.g, (int*)M.ls.swidth, &M.dint[4], e.vb);
}

__global__ __launch_bounds__(NT) void k_boundary_seg(const BMember* __restrict__ t,
                                                     const BMap* __restrict__ map) {
    const BMap e = map[blockIdx.x];
    const BMember& M = t[e.q];
    if (M.mode != FIM_LOCAL) return;
    boundary_rows(M.nA, M.ls.l2g, M.ls.g2l, M.g, M.bnd, &M.dint[2], e.vb);
}

void launch_structure_seg(const BMember* t, const BMap* rows, int nrows, const BMap* mem,
                          int nmem, int cell_stride, hipStream_t s) {
    if (nmem <= 0) return;
    k_struct_reset_seg<<<nmem, 64, 0, s>>>(t, mem);
    if (nrows <= 0) return;
    k_slice_width_seg<<<nrows, NT, 0, s>>>(t, rows);
    launch_pc_blocks_seg(t, rows, nrows, cell_stride, s);
    k_boundary_seg<<<nrows, NT, 0, s>>>(t, rows);
}

void launch_shrink(int nA, const int* l2g, const double* dp_abs, double eps,
                   const Graph& g, uint8_t* act, const int* flag,
                   hipStream_t s) {
    if (nA > 0) k_shrink<<<nblocks(nA), NT, 0, s>>>(nA, l2g, dp_abs, eps, g, act, flag);
}

// First-step initial set: the always-active cells and their m-layer
// neighbourhood (act must be cleared before).
__global__ __launch_bounds__(NT) void k_mark_seeds(int n, Graph g, uint8_t* __restrict__ lvl,
                                                   uint8_t* act) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool seed = (g.flags[i] & CF_AA) != 0;
    lvl[i] = seed ? 0 : 0xff;
    if (seed) act[i] = 1;
}

void launch_mark_seeds(int n, const Graph& g, int m, uint8_t* act, uint8_t* lvl,
                       hipStream_t s) {
    if (n <= 0) return;
    k_mark_seeds<<<nblocks(n), NT, 0, s>>>(n, g, lvl, act);
    ball_steps(n, g, m < MAX_LAYERS ? m : MAX_LAYERS, lvl, act, nullptr, s);
}

// Later steps: the support of the previous timestep plus the always-active
// cells.
__global__ __launch_bounds__(NT) void k_support(int n, const double* __restrict__ p,
                                                const double* __restrict__ pn, double eps,
                                                Graph g, uint8_t* __restrict__ act) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    act[i] = (fabs(p[i] - pn[i]) >= eps || (g.flags[i] & CF_AA)) ? 1 : 0;
}

void launch_support(int n, const double* p, const double* pn, double eps,
                    const Graph& g, uint8_t* act, hipStream_t s) {
    if (n > 0) k_support<<<nblocks(n), NT, 0, s>>>(n, p, pn, eps, g, act);
}

// Localized fracture cells: every fracture component (fracture cells
// connected through fracture-fracture connections) with an active cell
// becomes active as a whole.  Pass 1 flags the components that hold an
// active cell, pass 2 activates every cell of a flagged component; both
// run over the list of fracture cells only.
__global__ __launch_bounds__(NT) void k_frac_touch(int nf, const int* __restrict__ fcells,
                                                   const int* __restrict__ fcomp,
                                                   const uint8_t* __restrict__ act,
                                                   uint8_t* __restrict__ touch) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nf && act[fcells[q]]) touch[fcomp[q]] = 1;
}

__global__ __launch_bounds__(NT) void k_frac_close(int nf, const int* __restrict__ fcells,
                                                   const int* __restrict__ fcomp,
                                                   const uint8_t* __restrict__ touch,
                                                   uint8_t* __restrict__ act) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nf && touch[fcomp[q]]) act[fcells[q]] = 1;
}

void launch_frac_closure(int nf, const int* fcells, const int* fcomp, int ncomp,
                         uint8_t* touch, uint8_t* act, hipStream_t s) {
    if (nf <= 0) return;
    launch_fill_u8(touch, ncomp, 0, s);
    k_frac_touch<<<nblocks(nf), NT, 0, s>>>(nf, fcells, fcomp, act, touch);
    k_frac_close<<<nblocks(nf), NT, 0, s>>>(nf, fcells, fcomp, touch, act);
}

// Additive Algorithm 2: each cell takes the update of the first subdomain
// (in build order) that contains it.  Subdomain k's cells get owner k
// unless an earlier subdomain owns them; the lists are launched in build
// order, so no two threads of one launch race for a cell.
__global__ void k_set_owner(int cnt, const int* __restrict__ cells, int* __restrict__ owner,
                            int k) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < cnt && owner[cells[q]] < 0) owner[cells[q]] = k;
}

void launch_set_owner(int cnt, const int* cells, int* owner, int k, hipStream_t s) {
    if (cnt > 0) k_set_owner<<<nblocks(cnt), NT, 0, s>>>(cnt, cells, owner, k);
}

__global__ void k_copy_owned(int nA, const int* __restrict__ l2g, const int* __restrict__ owner,
                             int k, const double* __restrict__ src, double* __restrict__ dst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nA) {
        const int i = l2g[r];
        if (owner[i] == k) dst[i] = src[i];
    }
}

void launch_copy_owned(int nA, const int* l2g, const int* owner, int k, const double* src,
                       double* dst, hipStream_t s) {
    if (nA > 0) k_copy_owned<<<nblocks(nA), NT, 0, s>>>(nA, l2g, owner, k, src, dst);
}

// Algorithm 2: V_B^{k+1} = boundary(V_T) intersected with V_A^{k+1}.
__global__ __launch_bounds__(NT) void k_dd_boundary(int nA, const int* __restrict__ l2g,
                                                    const uint8_t* __restrict__ vt, Graph g,
                                                    uint8_t* __restrict__ bnd) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nA) return;
    const int i = l2g[r];
    uint8_t b = 0;
    for (int e = g.adj_ptr[i]; e < g.adj_ptr[i + 1]; e++)
        if (!vt[g.adj_nbr[e]]) { b = 1; break; }
    bnd[i] = b;
}

void launch_dd_boundary(int nA, const int* l2g, const uint8_t* vt,
                        const Graph& g, uint8_t* bnd, hipStream_t s) {
    if (nA > 0) k_dd_boundary<<<nblocks(nA), NT, 0, s>>>(nA, l2g, vt, g, bnd);
}

// Outer layer dB of a set: cells outside it adjacent to it.
__global__ __launch_bounds__(NT) void k_outer_layer(int nA, const int* __restrict__ l2g,
                                                    const uint8_t* __restrict__ in_set,
                                                    Graph g, uint8_t* outer) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nA) return;
    const int i = l2g[r];
    for (int e = g.adj_ptr[i]; e < g.adj_ptr[i + 1]; e++) {
        const int j = g.adj_nbr[e];
        if (!in_set[j]) outer[j] = 1;
    }
}

void launch_outer_layer(int nA, const int* l2g, const uint8_t* in_set,
                        const Graph& g, uint8_t* outer, hipStream_t s) {
    if (nA > 0) k_outer_layer<<<nblocks(nA), NT, 0, s>>>(nA, l2g, in_set, g, outer);
}

// max of v[idx[k]] over k < cnt into *out (single block, deterministic)
__global__ __launch_bounds__(NT) void k_gather_max(int cnt, const int* __restrict__ idx,
                                                   const double* __restrict__ v,
                                                   double* __restrict__ out) {
    double m[1] = {0.0};
    for (int k = threadIdx.x; k < cnt; k += NT) m[0] = fmax(m[0], v[idx[k]]);
    block_max<1>(m);
    if (threadIdx.x == 0) *out = m[0];
}

void launch_gather_max(int cnt, const int* idx, const double* v, double* out,
                       hipStream_t s) {
    k_gather_max<<<1, NT, 0, s>>>(cnt, idx, v, out);
}

// four cell classes of one iteration: bit 0 active, bit 1 boundary,
// bit 2 update >= eps (inactive cells keep 0)
__global__ __launch_bounds__(NT) void k_cell_classes(int nA, const int* __restrict__ l2g,
                                                     const uint8_t* __restrict__ bnd, int use_bnd,
                                                     const double* __restrict__ dp_abs, double eps,
                                                     uint8_t* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nA) return;
    const int i = l2g[r];
    out[i] = (uint8_t)(1 | ((use_bnd && bnd[i]) ? 2 : 0) | (dp_abs[i] >= eps ? 4 : 0));
}

void launch_cell_classes(int nA, const int* l2g, const uint8_t* bnd, bool use_bnd,
                         const double* dp_abs, double eps, uint8_t* out, hipStream_t s) {
    if (nA > 0)
        k_cell_classes<<<nblocks(nA), NT, 0, s>>>(nA, l2g, bnd, use_bnd ? 1 : 0, dp_abs, eps, out);
}

__global__ void k_scatter_flags(int cnt, const int* __restrict__ idx, uint8_t* flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt) flags[idx[k]] = 1;
}

void launch_scatter_flags(int cnt, const int* idx, uint8_t* flags, hipStream_t s) {
    if (cnt > 0) k_scatter_flags<<<nblocks(cnt), NT, 0, s>>>(cnt, idx, flags);
}

__global__ void k_copy_masked(int nA, const int* __restrict__ l2g,
                              const double* __restrict__ src, double* __restrict__ dst) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nA) {
        const int i = l2g[r];
        dst[i] = src[i];
    }
}

void launch_copy_masked(int nA, const int* l2g, const double* src, double* dst,
                        hipStream_t s) {
    if (nA > 0) k_copy_masked<<<nblocks(nA), NT, 0, s>>>(nA, l2g, src, dst);
}

struct SubTab {
    long co[MAX_SUBS];
    long oo[MAX_SUBS];
    int cn[MAX_SUBS];
    int on[MAX_SUBS];
};

// SUB_WG workgroups per subdomain; the values are >= 0, so their IEEE bit
// patterns order like the values and an integer atomic max combines the
// workgroups' maxima (order-independent).
constexpr int SUB_WG = 64;

__global__ void k_zero_f64(double* out, int n) {
    if ((int)threadIdx.x < n) out[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(NT) void k_sub_max(SubTab t, const int* __restrict__ cells,
                                                const int* __restrict__ outer,
                                                const double* __restrict__ last_dp,
                                                double* __restrict__ out) {
    const int k = blockIdx.x / SUB_WG, w = blockIdx.x % SUB_WG;
    const int step = SUB_WG * NT, q0 = w * NT + threadIdx.x;
    double m[1] = {0.0};
    for (int q = q0; q < t.cn[k]; q += step) m[0] = fmax(m[0], last_dp[cells[t.co[k] + q]]);
    for (int q = q0; q < t.on[k]; q += step) m[0] = fmax(m[0], last_dp[outer[t.oo[k] + q]]);
    block_max<1>(m);
    if (threadIdx.x == 0 && m[0] > 0.0)
        atomicMax((unsigned long long*)&out[k], (unsigned long long)__double_as_longlong(m[0]));
}

void launch_sub_max(int N, const DDSub* subs, const int* cells, const int* outer,
                    const double* last_dp, double* out, hipStream_t s) {
    if (N <= 0) return;
    SubTab t;
    for (int k = 0; k < N && k < MAX_SUBS; k++) {
        t.co[k] = subs[k].cells_off;
        t.cn[k] = subs[k].cells_n;
        t.oo[k] = subs[k].outer_off;
        t.on[k] = subs[k].outer_n;
    }
    const int nk = N < MAX_SUBS ? N : MAX_SUBS;
    k_zero_f64<<<1, MAX_SUBS, 0, s>>>(out, nk);
    k_sub_max<<<nk * SUB_WG, NT, 0, s>>>(t, cells, outer, last_dp, out);
}

} // namespace fimk
