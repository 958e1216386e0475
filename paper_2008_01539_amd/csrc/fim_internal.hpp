// Internal declarations shared by the HIP translation units of libfim.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "fim.h"

namespace fimk {

constexpr int WAVE = 64;        // CDNA wavefront
constexpr int SLICE = 64;       // rows per sliced-ELL slice (= one wave)
constexpr int NT = 256;         // threads per block of row kernels
constexpr int TILE = 4096;      // cells per block in compaction (256 x 16)
constexpr int MAX_LAYERS = 8;   // deepest neighbourhood the marker walks
constexpr int MAX_SUBS = 64;    // Algorithm 2 subdomains per timestep
constexpr int KB_NT = 256;      // threads per block of the Krylov kernels
constexpr int KB_MAXB = 1024;   // blocks per Krylov launch (grid-stride above)
constexpr int PC_DOF = 64;      // unknowns per fracture preconditioner block (at most)
// cells per fracture block: PC_DOF / b, but 20 for b = 2 (measured: on the
// two-phase DFN workloads 20-cell blocks need about as many BiCGStab
// iterations as 32-cell ones, and the product kernels read 5/8 of the
// inverse bytes)
constexpr int pc_cells(int b) { return b == 2 ? 20 : PC_DOF / b; }

// Fracture-block inverse store.  A block of R rows (N = R b unknowns) at
// element offset off keeps entry (unknown u = rr b + c, column j) at
//   off + ((j / K) R + rr) W + c K + j % K,  K = pc_group_cols(b), W = b K:
// the columns in groups of K, and inside a group the b K entries of one row
// contiguous (a multiple of 16 bytes, read as 4-float vectors by the
// thread of that row); the last group is padded with zeros.  Each fracture
// cell reserves b PC_DOF entries, so a block whose first cell has fracture
// ordinal f fits before the next block's first ordinal (>= f + R).
constexpr int pc_group_cols(int b) { return b == 2 ? 2 : 4; }
constexpr int pc_cell_stride(int b) { return b * PC_DOF; }

// per-cell flag bits
enum : uint8_t { CF_FRAC = 1, CF_PERF = 2, CF_AA = 4 };

struct DevFluid {
    int kind;
    double p_ref, rho_ref, c, mu;
    double rho_w, c_w, mu_w, rho_o, c_o, mu_o, swc, sor;
    double rs_b, p_b, bo_slope, bg_c, rho_osc, rho_gsc, rho_wsc, mu_g, span;
    double c_r, p_ref_rock, gravity;
};

// Static model data resident in HBM (structure of arrays).
struct Graph {
    int n;
    const int* adj_ptr;     // [n+1]
    const int* adj_nbr;     // [2 nc] neighbours, ascending per row
    const double* adj_T;    // [2 nc] transmissibility of that connection
    const double* pv;       // [n]
    const double* depth;    // [n]
    const uint8_t* flags;   // [n]
    const double* wi;       // [n] well index (0 if not perforated)
    const double* bhp;      // [n]
};

// Local (compacted) block system in sliced-ELL form with a fixed slice
// stride: slice s holds rows 64s..64s+63 in slots 64 wcap s .. 64 wcap
// (s+1) - 1 (wcap = the largest row width of the grid, max degree + 1);
// slot (row r, k) sits at 64 (wcap s + k) + (r - 64 s) for k < swidth[s];
// slot k = 0 is the diagonal block; padding slots below the slice width
// have col = r and zero value, slots at or past it are never read for
// arithmetic.  The fixed stride puts a slot's address one step from the
// row index (no slice-pointer load in front of the column loads).
struct LocalSys {
    const int* l2g;         // [nA]
    const int* g2l;         // [n], -1 = inactive
    const int* swidth;      // [nslices] slots per row in slice s
    int wcap;               // slice stride / 64
    int pad;
    int* col;               // [slots]
    double* J;              // [slots b b] FP64 Jacobian blocks
    double* F;              // [nA b]
};
__host__ __device__ inline long slot_of(const LocalSys& ls, int r, int k) {
    return ((long)(r / SLICE) * ls.wcap + k) * SLICE + (r % SLICE);
}

// Scalars of the BiCGStab iteration, recorded by block 0 of each kernel
// for the kernels that follow and for the host.
struct KScal {
    double rho_hist[2];     // rho_i at slot i & 1
    double alpha, omega, rr;
    int done, iters, breakdown, pad;
};

// Newton-iteration status words (one readback per iteration).
struct NStat {
    double dp_max, ds_max;
    int nswitch, nonfinite;
    int n_active, n_bnd, is_expand, n_next;
};

// ------------------------------------------------------------ launches
// sets / compaction (fim_sets.hip)
void launch_fill_u8(uint8_t* a, int n, uint8_t v, hipStream_t s);
void launch_fill_i32(int* a, int n, int v, hipStream_t s);
void launch_fill_f64(double* a, long n, double v, hipStream_t s);
// the iteration's status words (ns may be null: dint only) into mapped
// pinned host memory, one launch instead of two copies
void launch_status_out(const NStat* ns, const int* dint, NStat* ons, int* oint, hipStream_t s);
void launch_compact(const uint8_t* act, int n, int* blk_cnt, int* l2g,
                    int* g2l, int* n_out, hipStream_t s);
// also writes the number of blocks of the local matrix (diagonal included)
void launch_structure(int nA, const int* l2g, const int* g2l, const Graph& g,
                      int* swidth, int* nnzb, hipStream_t s);
void launch_boundary(int nA, const int* l2g, const int* g2l, const Graph& g,
                     uint8_t* bnd, int* count, hipStream_t s);
// lvl: n bytes of scratch (graph distance to the nearest seed)
void launch_mark_expand(int nA, const int* l2g, const uint8_t* bnd,
                        const double* dp_abs, double eps, int m,
                        const Graph& g, uint8_t* act, uint8_t* act2,
                        int* flag, uint8_t* lvl, hipStream_t s);
void launch_shrink(int nA, const int* l2g, const double* dp_abs, double eps,
                   const Graph& g, uint8_t* act, const int* flag,
                   hipStream_t s);
void launch_mark_seeds(int n, const Graph& g, int m, uint8_t* act, uint8_t* lvl,
                       hipStream_t s);
// residual-based set: act = {err_i >= tol} and its m-layer neighbourhood on
// all n cells; *count += number of cells with err_i >= tol
void launch_mark_resid(int n, const double* err, double tol, int m, const Graph& g,
                       uint8_t* act, int* count, uint8_t* lvl, hipStream_t s);
void launch_support(int n, const double* p, const double* pn, double eps,
                    const Graph& g, uint8_t* act, hipStream_t s);
// localized fracture cells: activate every fracture component that holds
// an active cell (fcells: the nf fracture cells, fcomp their components
// 0..ncomp-1, touch: ncomp bytes of scratch)
void launch_frac_closure(int nf, const int* fcells, const int* fcomp, int ncomp,
                         uint8_t* touch, uint8_t* act, hipStream_t s);
// additive Algorithm 2: owner[c] = k for the cells of a subdomain list
// that have no owner yet; dst[i] = src[i] for the rows of a local system
// whose cell is owned by k
void launch_set_owner(int cnt, const int* cells, int* owner, int k, hipStream_t s);
void launch_copy_owned(int nA, const int* l2g, const int* owner, int k, const double* src,
                       double* dst, hipStream_t s);
void launch_dd_boundary(int nA, const int* l2g, const uint8_t* vt,
                        const Graph& g, uint8_t* bnd, hipStream_t s);
void launch_outer_layer(int nA, const int* l2g, const uint8_t* in_set,
                        const Graph& g, uint8_t* outer, hipStream_t s);
void launch_gather_max(int cnt, const int* idx, const double* v, double* out,
                       hipStream_t s);
void launch_scatter_flags(int cnt, const int* idx, uint8_t* flags, hipStream_t s);
void launch_cell_classes(int nA, const int* l2g, const uint8_t* bnd, bool use_bnd,
                         const double* dp_abs, double eps, uint8_t* out, hipStream_t s);
void launch_copy_masked(int nA, const int* l2g, const double* src, double* dst,
                        hipStream_t s);

// Algorithm 2 subdomain k: cells sd_cells[cells_off .. +cells_n) (= V_A^k,
// ascending) and its outer layer sd_outer[outer_off .. +outer_n)
struct DDSub {
    long cells_off;
    int cells_n;
    long outer_off;
    int outer_n;
};
// out[k] = max of last_dp over V_A^k and its outer layer, k < N <= MAX_SUBS
void launch_sub_max(int N, const DDSub* subs, const int* cells, const int* outer,
                    const double* last_dp, double* out, hipStream_t s);

// physics (fim_assemble.hip)
void launch_accumulation(int fk, int n, const double* u, const int8_t* st,
                         const Graph& g, const DevFluid& f, double* M,
                         hipStream_t s);
void launch_assemble(int fk, int nA, const LocalSys& ls, const Graph& g,
                     const DevFluid& f, const double* u, const int8_t* st,
                     const double* Mn, double inv_dt, hipStream_t s);
// e_i = dt max_c |R_{i,c}| / (V_i rho_c) on all n cells
void launch_resid_err(int fk, int n, const Graph& g, const DevFluid& f, const double* u,
                      const int8_t* st, const double* Mn, double dt, double* err,
                      hipStream_t s);
void launch_precond(int b, bool fp32, int nA, const LocalSys& ls,
                    double* dinv, void* At, hipStream_t s);

// Krylov (fim_krylov.hip)
struct KrylovBufs {
    void* x; void* r; void* rh; void* p[2]; void* v[2]; void* sv; void* t;
    double* x64; double* rir; KScal* sc;
    double* xprev;          // x64 before the last FP32 pass (its undo)
    // per-block partial dot products (part_ir 2 per block, the others 4)
    double* part_ir; double* part_a; double* part_b; double* part_c;
    const double* dinv; const void* At;
    // fracture-block preconditioner (pcM NULL: block Jacobi only)
    const int* pcinfo; const int* pcoff; const float* pcM;   // FP32 inverses
    int pcdec;              // unknowns decoupled inside the blocks (FIM_PC_FRACTURE)
    int pad_;
};
// workgroups of a Krylov launch over nA rows: one per 256-row tile, at most
// cap (the kernels loop over further tiles)
int krylov_grid(int nA, int cap);

// One model's share of a (batched) Krylov launch.  A launch covers the
// blocks of every participating model; block q belongs to model
// blk_seg[q] and is that model's block q - blk0 of nblk.  A model sees the
// same block partition, the same per-block partial sums and the same
// reduction order alone and in a batch, so its results are identical.
struct KSeg {
    LocalSys ls;
    KrylovBufs kb;
    int nA;
    int blk0, nblk;
    int active;
    double tol2;       // stop when |r|^2 <= tol2
    double bnorm2;     // |b~|^2 of the refinement pass (breakdown scale)
    int maxit;
    int pad;
};

// r64 = -F - J x64, b~ = D^{-1} r64, Krylov initialisation; part_ir holds
// (|r64|^2, |b~|^2) per block
// solo: the launch covers one model (segs[0]); its blocks then skip the
// block-to-model lookup
void launch_ir_residual(int b, bool fp32, bool solo, const KSeg* segs, const int* blk_seg,
                        int nblk_total, bool x_zero, hipStream_t s);
// which: 0 = kernel P (x, r update of iteration it-1; p and v = A p of it),
// 1 = kernel S (s = r - alpha v, t = A s); it = iteration index (same for
// every model of the launch)
// pc: some model of the launch has fracture blocks (the kernels then apply
// their inverses to the product on the fracture rows)
// ev0/ev1: optional events stamped with the kernel's own start and end
// rec (kernel S only, optional): one SegStatus per model of the launch with
// the Krylov status after this kernel (rr, done, iters, breakdown; the
// refinement sums zero); may be the device address of coherent pinned host
// memory
struct SegStatus;
// wide (FP32 with fracture blocks only): the launch has more workgroups
// than two per CU; a variant with three resident per CU runs it
// pc: the members' fracture blocks (0 none, 1 coupled, 2 the unknowns
// decoupled; members without blocks use block Jacobi in any launch)
void launch_bicg_part(int which, int b, bool fp32, bool solo, int pc, const KSeg* segs,
                      const int* blk_seg, int nblk_total, int it, hipStream_t s,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                      SegStatus* rec = nullptr, bool wide = false);
void launch_ir_accumulate(int b, bool fp32, bool solo, const KSeg* segs, const int* blk_seg,
                          int nblk_total, hipStream_t s);

struct SegStatus {
    double rir2, bnorm2;
    double rr;              // BiCGStab |r|^2 at the last completed iteration
    int done, iters, breakdown, pad;
};
// out: nseg records; may be the device address of coherent pinned host memory
void launch_seg_status(const KSeg* segs, int nseg, SegStatus* out, hipStream_t s);
void launch_copy_f64(double* dst, const double* src, long n, hipStream_t s);

// fracture-block preconditioner (fim_fracpc.hip)
// funit[cell] (fracture cells) = unit << 8 | cap_units: the cell's unit (its
// position inside its fracture, in cell index order, divided by the unit
// length of the fracture) and the most units one block may hold; blocks
// split a fracture's run of rows at unit boundaries into about equal parts.
// list: (first row, rows) of each multi-row block (room for nA / 2
// blocks); cnt[0] = sum over them of rows^2, cnt[1] = their number
void launch_pc_blocks(int nA, const int* l2g, const int* frac_id, const int* ford,
                      const int* funit, int cell_stride, int* pcinfo, int* pcoff, int* list,
                      int* cnt, hipStream_t s);
// At: the scaled blocks in the Krylov precision (fp32: float, else double);
// grid single-wave workgroups share the listed blocks
// dec: one inverse per unknown over the block's cells (the unknowns
// decoupled), stored as the block's rows x rows columns of the layout
void launch_pc_invert(int b, bool fp32, int grid, const LocalSys& ls, const void* At,
                      const int* list, const int* cnt, const int* pcoff, float* pcM,
                      bool dec, hipStream_t s);
// one system of a batched inversion (device table entry)
struct PcSeg {
    LocalSys ls;
    const void* At;
    const int* list;
    const int* cnt;
    const int* pcoff;
    float* pcM;
};
// the blocks of nseg systems (same b, Krylov precision and fracture-block
// mode dec) in one launch of grid single-wave workgroups; pref: nseg + 1
// ints of device scratch
void launch_pc_invert_batch(int b, bool fp32, int grid, const PcSeg* segs, int nseg, int* pref,
                            bool dec, hipStream_t s);

// update (fim_update.hip)
void launch_update(int fk, int nA, const int* l2g, const double* x64,
                   double* u, int8_t* st, int n, const DevFluid& f,
                   double ds_max, double* dp_abs, double* part, NStat* ns,
                   hipStream_t s,
                   const int* owner = nullptr, int own_k = 0);
void launch_copy_state(int b, int n, const double* src, const int8_t* ssrc,
                       double* dst, int8_t* sdst, hipStream_t s);

// ------------------------------------------------ batched Newton iteration
// One member of a batched Newton iteration as the segmented kernels see it
// (a device table of these, rewritten by the host for each phase of a
// batched call): its graph, fluid, state, local system and set buffers,
// and its current n_A.  Members share the block size and Krylov precision.
struct BMember {
    LocalSys ls;
    Graph g;
    DevFluid f;
    double* u;
    int8_t* st;
    double* Mn;
    double* un;             // state and accumulation at the start of the step
    int8_t* stn;
    uint8_t* supp;          // support of the last converged step
    double inv_dt, dt, ds_max;
    double* dinv;
    void* At;
    double* x64;
    double* dp_abs;
    double* part;           // update partials (4 per row workgroup)
    NStat* ns;
    uint8_t* act;
    uint8_t* bnd;
    uint8_t* lvl;
    int* dint;              // [0] expand flag / unconverged count, [1] n_next,
                            // [2] boundary count, [4] matrix blocks, [5..6] fracture blocks
    int* blk;               // compaction tile counts
    double* last_dp;        // residual error measure (FIM_RESID)
    double eps_loc, eps_res;
    const int* frac_id;     // fracture blocks (null: none)
    const int* ford;
    const int* funit;
    int* pcinfo;
    int* pcoff;
    int* pclist;
    int n, nA, mode, layers;
    // per phase: begin = starts a timestep (0 no; 1 act = supp; 2 act = the
    // always-active cells and their layers-layer neighbourhood; 3 act = all
    // cells; 4 keep act), compact = compacts act, commit = the step
    // converged (its support into supp)
    int begin, compact, commit, pad;
};
// workgroup -> (member, the member's own workgroup index)
struct BMap {
    int q, vb;
};
// the workgroup maps of a batched phase from three exclusive prefix arrays
// of K + 1 ints (row, cell, tile workgroups of each member); most: the
// largest of the three totals
void launch_build_maps(const int* pref, int K, int most, BMap* rows, BMap* cells, BMap* tiles,
                       BMap* mem, hipStream_t s);
// Segmented launches: nblk workgroups, map[blockIdx.x] names the member and
// its workgroup.  Row launches cover each member's n_A rows (NT per
// workgroup), cell launches its n cells, tile launches its n cells in
// TILE-cell tiles, member launches one workgroup per member.
void launch_assemble_seg(int fk, const BMember* t, const BMap* rows, int nblk, hipStream_t s);
// (also zeroes each member's x64 rows)
void launch_precond_seg(int b, bool fp32, const BMember* t, const BMap* rows, int nblk,
                        hipStream_t s);
// the FIM_RESID members' error measure into last_dp (cell launch)
void launch_resid_err_seg(int fk, const BMember* t, const BMap* cells, int nblk, hipStream_t s);
// update + per-member reduction (one workgroup per member in mem); each
// member's update workgroup count is nblocks(n_A) (its own partials)
void launch_update_seg(int fk, const BMember* t, const BMap* rows, int nblk, const BMap* mem,
                       int nmem, hipStream_t s);
// Algorithm 1 expand / shrink (FIM_LOCAL members) and the residual-based
// marking (FIM_RESID members); layers: the largest member layer count
void launch_sets_seg(int fk, const BMember* t, const BMap* rows, int nrows, const BMap* cells,
                     int ncells, const BMap* mem, int nmem, int layers, bool any_resid,
                     hipStream_t s);
// compaction of act (the members with compact set)
void launch_compact_seg(const BMember* t, const BMap* tiles, int ntiles, hipStream_t s);
// timestep start of the members with begin set: u^n, status^n and the
// accumulation at u^n, the first active flags (begin 1 - 3), then the
// neighbour layers of begin-2 members (layers: their largest count)
void launch_begin_seg(int fk, const BMember* t, const BMap* cells, int ncells, int layers,
                      hipStream_t s);
// (fim_sets.hip) layers passes of the neighbourhood marking over the
// members' own layer counts
void launch_ball_steps_seg(const BMember* t, const BMap* cells, int ncells, int layers,
                           hipStream_t s);
// the support of the converged steps (members with commit set)
void launch_support_seg(const BMember* t, const BMap* cells, int ncells, hipStream_t s);
// each member's NStat and dint[0..3] into out (pinned host, nmem records)
struct BStatus {
    NStat ns;
    int dint[4];
};
void launch_status_seg(const BMember* t, const BMap* mem, int nmem, BStatus* out, hipStream_t s);
// structure of the new local systems (slice widths, fracture blocks of the
// members that have them) and, for FIM_LOCAL members, the boundary V_B
void launch_structure_seg(const BMember* t, const BMap* rows, int nrows, const BMap* mem,
                          int nmem, int cell_stride, hipStream_t s);
// (fim_fracpc.hip) the fracture-block layout of the members with blocks
void launch_pc_blocks_seg(const BMember* t, const BMap* rows, int nrows, int cell_stride,
                          hipStream_t s);

} // namespace fimk
