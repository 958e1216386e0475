// Host driver and C ABI of libfim: model residency in HBM, the Newton
// iteration (Section 4.1), the localized Newton state machine
// (Algorithm 1), the adaptive nonlinear domain decomposition
// (Algorithm 2), the residual-based localization the paper compares
// against (Sections 1 and 4.2), the iterative-refinement Krylov driver and
// the inspection entry points.  All arithmetic of the path runs in the kernels; the host
// only sequences launches and reads one small status record per Newton
// iteration (plus one per block of Krylov iterations).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fim_internal.hpp"

using namespace fimk;

// Optional event profiler: hipEvent pairs on the model's stream around each
// kernel (or kernel group), read back at the next synchronisation.
enum { PK_ASSEMBLE, PK_PRECOND, PK_IR, PK_BICG_A, PK_BICG_B, PK_UPDATE, PK_SETS, PK_SETUP,
       PK_PCINV, PK_N };
static const char* const kPkName[PK_N] = {"assemble", "precond", "ir_residual", "bicg_spmv_p",
                                          "bicg_spmv_s", "update", "sets_compact",
                                          "step_setup", "frac_invert"};
struct ProfRec {
    int k;
    hipEvent_t a, b;
    double rows;
    bool matrix;   // launch works on the current local matrix (nnzb known later)
    int tag;       // BiCGStab iteration within a block of queued iterations, else -1
};
struct Prof {
    bool on = false;
    std::vector<ProfRec> pend;
    std::vector<hipEvent_t> pool;
    double ms[PK_N] = {};
    double rows[PK_N] = {};
    double nnzb[PK_N] = {};
    double aux[PK_N] = {};
    long cnt[PK_N] = {};
};


// Tables of a (batched) Krylov launch: per-model descriptors and the
// block -> model map, in device memory, plus pinned status records.
struct SolveTable {
    KSeg* dsegs = nullptr;
    int* dblk = nullptr;
    // [6][cap]: refinement status, then 2 x 2 Krylov slots, in pinned host
    // memory that k_seg_status writes directly (hstat_dev: its device
    // address), so no copy runs between the Krylov kernels
    SegStatus* hstat_dev = nullptr;
    SegStatus* hstat = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    // batched fracture-block inversion: [2][cap] systems (FP32, FP64 Krylov)
    // and [2][cap + 1] running block counts
    PcSeg* dpc = nullptr;
    int* dpref = nullptr;
    // pinned staging of the uploads ([2][cap] descriptors, [2][cap * KB_MAXB]
    // block map): asynchronous copies; the host rewrites them only after a
    // synchronisation that follows the previous copy
    KSeg* hsegs = nullptr;
    int* hblk = nullptr;
    int cap = 0;
};

// Scratch of the allocation-free Newton iteration (fim_newton_step_noalloc):
// one static device array per GPU that the library runs on, held until
// the process ends.  Host code never passes the array's name to a kernel
// (in host code it is a host-side stand-in, not a device address): the
// address comes from hipGetSymbolAddress, taken once per device with that
// device current and kept per device.  Layout (bytes, 256-aligned parts):
// the Krylov partial sums (14 KB_MAXB doubles), the Krylov scalars, the two
// launch descriptors of a one-model solve and its (unread) block map, the
// compaction tile counts and the update's per-block partials, sized for
// models of at most NA_MAX_CELLS cells.
constexpr int NA_MAX_CELLS = 1 << 22;
constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t NA_OFF_PART = 0;
constexpr size_t NA_OFF_SC = NA_OFF_PART + na_align(14 * KB_MAXB * sizeof(double));
constexpr size_t NA_OFF_SEGS = NA_OFF_SC + na_align(sizeof(KScal));
constexpr size_t NA_OFF_BMAP = NA_OFF_SEGS + na_align(2 * sizeof(KSeg));
constexpr size_t NA_OFF_TILES = NA_OFF_BMAP + na_align(2 * KB_MAXB * sizeof(int));
constexpr size_t NA_OFF_UPART =
    NA_OFF_TILES + na_align(((size_t)NA_MAX_CELLS / TILE + 2) * sizeof(int));
constexpr size_t NA_SCRATCH_BYTES =
    NA_OFF_UPART + na_align(4 * ((size_t)NA_MAX_CELLS / NT + 2) * sizeof(double));
static __device__ __align__(256) char scratch[NA_SCRATCH_BYTES];
static_assert(sizeof(KScal) % sizeof(int) == 0, "KScal is cleared as ints");

constexpr int NA_MAX_DEV = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[NA_MAX_DEV] = {};
static bool g_scratch_done[NA_MAX_DEV] = {};
static std::string g_scratch_err[NA_MAX_DEV];

// The scratch address on the current device (looked up once per device);
// null with *why set when it is not available.
static char* scratch_address(int dev, std::string* why) {
    if (dev < 0 || dev >= NA_MAX_DEV) {
        *why = "device ordinal out of range for the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p) {
            g_scratch_ptr[dev] = (char*)p;
        } else {
            g_scratch_err[dev] = std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e);
        }
        g_scratch_done[dev] = true;
    }
    if (!g_scratch_ptr[dev]) *why = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}

struct fim_model {
    int n = 0, nconn = 0, B = 1, fk = 1;
    fim_options o{};
    DevFluid f{};
    hipStream_t s = nullptr;
    bool own_stream = false;
    hipEvent_t sync_ev = nullptr;   // see spin_sync
    Graph g{};
    // static data
    int *adj_ptr = nullptr, *adj_nbr = nullptr;
    double *adj_T = nullptr, *pv = nullptr, *depth = nullptr, *wi = nullptr, *bhp = nullptr;
    uint8_t* flags = nullptr;
    int max_deg = 0;
    // state
    double *u = nullptr, *un = nullptr, *Mn = nullptr, *dp_abs = nullptr, *last_dp = nullptr;
    int8_t *st = nullptr, *stn = nullptr;
    uint8_t *act = nullptr, *act2 = nullptr, *supp = nullptr, *bnd = nullptr, *vt = nullptr,
            *outer = nullptr;
    uint8_t* lvl = nullptr;         // neighbourhood marking: distance to the nearest seed
    // local system
    int *l2g = nullptr, *g2l = nullptr, *swidth = nullptr, *blk = nullptr;
    int *col = nullptr;
    double *J = nullptr, *F = nullptr, *dinv = nullptr;
    void* At = nullptr;
    long slot_cap = 0;
    // fracture-block preconditioner (use_pc false: block Jacobi only)
    bool use_pc = false;
    int pc_cap = 0;                 // rows per block
    bool pc_dec = false;            // unknowns decoupled inside the blocks
    int* funit = nullptr;           // fracture cells: unit << 8 | units per block
    int pc_grid = KB_MAXB;          // Krylov workgroups with fracture blocks (2 per CU)
    int pc_grid_wide = KB_MAXB;     // the same in the three-per-CU FP32 variant
    int *frac_id = nullptr, *ford = nullptr, *pcinfo = nullptr, *pcoff = nullptr;
    int* pclist = nullptr;          // multi-row blocks: (first row, rows) pairs
    int pc_inv_grid = 0;            // workgroups of the inversion launch
    int pc_nfc = 0;                 // fracture cells (inverse store size)
    int cus = 256;                  // compute units of the device
    float* pcM = nullptr;           // FP32 inverses
    // Krylov
    double *x64 = nullptr, *xprev = nullptr, *rir = nullptr, *part = nullptr;
    double* part_ir = nullptr;   // Krylov partials: 14 x KB_MAXB
    double* hpart = nullptr;     // pinned copy of the refinement partials
    void* kvec = nullptr;   // 9 vectors of nA b elements in the Krylov precision
    KScal* sc = nullptr;
    NStat* ns = nullptr;
    int* dint = nullptr;    // [0] expand flag, [1] n_next, [2] boundary count
    double* dsub = nullptr; // Algorithm 2 per-subdomain maxima
    // pinned host mirrors
    KScal* hsc = nullptr;
    NStat* hns = nullptr;
    int* hint = nullptr;
    NStat* hns_dev = nullptr;   // device addresses of hns / hint (mapped)
    int* hint_dev = nullptr;
    double* hsub = nullptr;
    // Algorithm 2 storage
    int *sd_cells = nullptr, *sd_outer = nullptr;
    long sd_cap = 0, sd_used = 0, ob_cap = 0, ob_used = 0;
    std::vector<DDSub> subs;
    int dd_phase = 0, dd_next = 0, dd_sweeps = 0, dd_k = 0;
    bool dd_valid = false;          // vt holds V_T of an Algorithm 2 timestep
    // additive Algorithm 2 (FIM_DD_ADD): the first subdomain of each cell,
    // one workspace per subdomain solved at once (a clone that shares the
    // model's static data and state and owns its local-system buffers), the
    // solve table of the batched subdomain solves
    int* dd_owner = nullptr;
    std::vector<fim_model*> dd_clones;
    SolveTable dd_tab;
    bool is_clone = false;
    // step state machine
    bool in_step = false, have_history = false, full_ready = false;
    double ew_fprev = 0.0, ew_eta = 0.0;   // forcing term: last |F| and eta of the step
    // Algorithm 2's phase 2: the forcing term per subdomain (its own last
    // |F| and eta) and the subdomain being solved (-1: none)
    std::vector<double> dd_ew_f, dd_ew_eta;
    int dd_cur = -1;
    fim_model* ew_owner = nullptr;   // a subdomain workspace: the model whose sequences it uses
    double step_dt = 0.0;
    int step_mode = 0, nu = 0, nA = 0, nB = 0;
    bool is_expand = true;
    double sum_active = 0.0;
    int max_active = 0, step_kry = 0;
    int last_kry = 0, last_refine = 0, last_fallback = 0;
    double last_relres = 0.0;
    bool inspect_ready = false;
    int cur_nnzb = 0;   // blocks of the current local matrix (profiling)
    double cur_pcn2 = 0.0;   // sum of N^2 over its fracture blocks (profiling)
    bool flags_on = false;
    // localized fracture cells (some fracture cell not always active):
    // Algorithm 1's sets are closed under fracture components; fcells
    // lists the fracture cells, fcomp their components, ftouch one flag
    // per component
    bool fclose = false;
    int nfcell = 0, ncomp = 0;
    int *fcells = nullptr, *fcomp = nullptr;
    uint8_t* ftouch = nullptr;
    // auto_cut: the state, phase status and support set on entry to
    // fim_solve_timestep, restored when the last substep fails
    double* usave = nullptr;
    int8_t* stsave = nullptr;
    uint8_t* suppsave = nullptr;
    SolveTable solo;
    // allocation-free Newton iterations (fim_newton_step_noalloc): the
    // kernels' partial sums, Krylov scalars, compaction tile counts and
    // launch descriptors live in the per-device static scratch array;
    // nat is the solve table of those calls (device parts in the scratch
    // array, pinned host parts allocated with the model)
    int dev = 0;
    char* scratch = nullptr;        // this device's scratch address (null: unavailable)
    SolveTable nat;
    bool noalloc = false;           // inside fim_newton_step_noalloc
    size_t bytes = 0;   // device bytes held
    uint8_t* classes = nullptr;   // per-cell classes of the last iteration
    Prof prof;
    std::string err;
};

static hipEvent_t ev_take(fim_model* m) {
    if (!m->prof.pool.empty()) {
        hipEvent_t e = m->prof.pool.back();
        m->prof.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

static int pbeg(fim_model* m, int k, int tag = -1) {
    if (!m->prof.on) return -1;
    const bool mat = k == PK_ASSEMBLE || k == PK_PRECOND || k == PK_IR || k == PK_BICG_A ||
                     k == PK_BICG_B;
    ProfRec r{k, ev_take(m), ev_take(m), 0.0, mat, tag};
    (void)hipEventRecord(r.a, m->s);
    m->prof.pend.push_back(r);
    return (int)m->prof.pend.size() - 1;
}

// record for a launch whose events the dispatch stamps (hipExtLaunchKernel)
static int pbeg_ext(fim_model* m, int k, int tag) {
    if (!m->prof.on) return -1;
    const bool mat = k == PK_BICG_A || k == PK_BICG_B;
    ProfRec r{k, ev_take(m), ev_take(m), 0.0, mat, tag};
    m->prof.pend.push_back(r);
    return (int)m->prof.pend.size() - 1;
}

static void pend(fim_model* m, int idx, double rows) {
    if (idx < 0) return;
    ProfRec& r = m->prof.pend[idx];
    r.rows = rows;
    (void)hipEventRecord(r.b, m->s);
}

// after a stream synchronisation; BiCGStab records tagged >= keep_tag were
// queued past convergence (the kernels returned at once) and are dropped
static void pflush(fim_model* m, int keep_tag = INT_MAX) {
    if (!m->prof.on) return;
    for (const ProfRec& r : m->prof.pend) {
        if (r.tag < keep_tag) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                m->prof.ms[r.k] += ms;
                m->prof.cnt[r.k] += 1;
                m->prof.rows[r.k] += r.rows;
                // matrix launches: blocks of the local matrix and entries of
                // the fracture-block inverses
                if (r.matrix) {
                    m->prof.nnzb[r.k] += m->cur_nnzb;
                    m->prof.aux[r.k] += m->cur_pcn2;   // the product kernels apply them
                }
            }
        }
        m->prof.pool.push_back(r.a);
        m->prof.pool.push_back(r.b);
    }
    m->prof.pend.clear();
}

#define HIPX(call)                                                           \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) {                                              \
            m->err = std::string(#call) + ": " + hipGetErrorString(e_);      \
            return FIM_E_HIP;                                                \
        }                                                                    \
    } while (0)

#define TRY(x)                                                               \
    do {                                                                     \
        fim_status r_ = (x);                                                 \
        if (r_ != FIM_OK) return r_;                                         \
    } while (0)

static fim_status dalloc(fim_model* m, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) m->bytes += bytes;
    if (e != hipSuccess) {
        m->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e);
        *p = nullptr;
        return FIM_E_NOMEM;
    }
    return FIM_OK;
}

template <typename P>
static fim_status dal(fim_model* m, P** p, size_t count) {
    return dalloc(m, (void**)p, count * sizeof(P));
}


// Waits for an event by polling rather than sleeping.  These waits sit
// between dependent launches on the host's critical path (status checks of
// the Newton and Krylov loops), where an interrupt-driven wake-up leaves the
// GPU idle for tens of microseconds.
static hipError_t spin_event(hipEvent_t e) {
    for (;;) {
        const hipError_t r = hipEventQuery(e);
        if (r != hipErrorNotReady) return r;
    }
}
// All work queued on s so far, through the model's own event
static hipError_t spin_sync(fim_model* m, hipStream_t s) {
    const hipError_t r = hipEventRecord(m->sync_ev, s);
    return r == hipSuccess ? spin_event(m->sync_ev) : r;
}

static fim_status sync_read(fim_model* m, void* host, const void* dev, size_t bytes,
                            int keep_tag = INT_MAX) {
    HIPX(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, m->s));
    HIPX(spin_sync(m, m->s));
    pflush(m, keep_tag);
    return FIM_OK;
}

static KrylovBufs kbufs(fim_model* m, bool fp32) {
    KrylovBufs kb;
    const size_t vb = (size_t)m->n * m->B * (fp32 ? 4 : 8);
    char* base = (char*)m->kvec;
    kb.x = base + 0 * vb;
    kb.r = base + 1 * vb;
    kb.rh = base + 2 * vb;
    kb.p[0] = base + 3 * vb;
    kb.p[1] = base + 4 * vb;
    kb.v[0] = base + 5 * vb;
    kb.v[1] = base + 6 * vb;
    kb.sv = base + 7 * vb;
    kb.t = base + 8 * vb;
    kb.x64 = m->x64;
    kb.xprev = m->xprev;
    kb.rir = m->rir;
    kb.sc = m->sc;
    kb.part_ir = m->part_ir;                 // 2 per block
    kb.part_a = m->part_ir + 2 * KB_MAXB;    // 4 per block
    kb.part_b = m->part_ir + 6 * KB_MAXB;
    kb.part_c = m->part_ir + 10 * KB_MAXB;
    kb.dinv = m->dinv;
    kb.At = m->At;
    kb.pcinfo = m->pcinfo;
    kb.pcoff = m->pcoff;
    kb.pcM = m->use_pc ? m->pcM : nullptr;
    kb.pcdec = m->pc_dec ? 1 : 0;
    return kb;
}

static LocalSys lsys(fim_model* m) {
    LocalSys ls;
    ls.l2g = m->l2g;
    ls.g2l = m->g2l;
    ls.swidth = m->swidth;
    ls.wcap = m->max_deg + 1;
    ls.pad = 0;
    ls.col = m->col;
    ls.J = m->J;
    ls.F = m->F;
    return ls;
}

// ---------------------------------------------------------------- pieces
// compaction of m->act into l2g/g2l; n_A lands in dint[1]
static void compact(fim_model* m) {
    launch_compact(m->act, m->n, m->blk, m->l2g, m->g2l, &m->dint[1], m->s);
}

static fim_status read_int(fim_model* m) {
    return sync_read(m, m->hint, m->dint, 4 * sizeof(int));
}

static fim_status structure(fim_model* m) {
    launch_structure(m->nA, m->l2g, m->g2l, m->g, m->swidth, &m->dint[4], m->s);
    if (m->use_pc)
        launch_pc_blocks(m->nA, m->l2g, m->frac_id, m->ford, m->funit, pc_cell_stride(m->B),
                         m->pcinfo, m->pcoff, m->pclist, &m->dint[5], m->s);
    return FIM_OK;
}

static void table_free(SolveTable& t) {
    for (hipEvent_t& e : t.ev)
        if (e) (void)hipEventDestroy(e);
    if (t.dsegs) (void)hipFree(t.dsegs);
    if (t.dblk) (void)hipFree(t.dblk);
    if (t.dpc) (void)hipFree(t.dpc);
    if (t.dpref) (void)hipFree(t.dpref);
    if (t.hstat) (void)hipHostFree(t.hstat);
    if (t.hsegs) (void)hipHostFree(t.hsegs);
    if (t.hblk) (void)hipHostFree(t.hblk);
    t = SolveTable();
}

// the pinned host parts and events of a solve table
static fim_status table_alloc_host(fim_model* m, SolveTable& t, int cap) {
    t.cap = cap;
    if (hipHostMalloc((void**)&t.hsegs, 2 * cap * sizeof(KSeg)) != hipSuccess ||
        hipHostMalloc((void**)&t.hblk, (size_t)2 * cap * KB_MAXB * sizeof(int)) != hipSuccess) {
        m->err = "hipHostMalloc failed";
        return FIM_E_NOMEM;
    }
    if (hipHostMalloc((void**)&t.hstat, 6 * cap * sizeof(SegStatus),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void**)&t.hstat_dev, t.hstat, 0) != hipSuccess) {
        m->err = "pinned status buffer not available";
        return FIM_E_NOMEM;
    }
    for (hipEvent_t& e : t.ev) HIPX(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return FIM_OK;
}

static fim_status table_alloc(fim_model* m, SolveTable& t, int cap) {
    TRY(table_alloc_host(m, t, cap));
    TRY(dal(m, &t.dpc, (size_t)2 * cap));
    TRY(dal(m, &t.dpref, (size_t)2 * (cap + 1)));
    TRY(dal(m, &t.dsegs, (size_t)2 * cap));
    TRY(dal(m, &t.dblk, (size_t)2 * cap * KB_MAXB));
    return FIM_OK;
}

// per-model state of one linear solve
struct SolveItem {
    fim_model* m;
    bool fp32;
    bool done_outer;
    bool active;
    double rir2, bnorm2, fnorm2, target2, tol2;
    int passes, kry, fallback;
};

// A group = the models of one Krylov precision; region g of the tables
// (g = 0: FP32, g = 1: FP64).
struct Group {
    std::vector<int> idx;   // items in this group
    int nblk = 0;
    int pc = 0;             // fracture blocks of the models that have them:
                            // 0 none, 1 coupled, 2 the unknowns decoupled
    bool wide = false;      // FP32 with fracture blocks, more tiles than 2 per CU
};

static fim_status upload_group(fim_model* lead, SolveTable& t, int g, Group& G,
                               std::vector<SolveItem>& items, hipStream_t s) {
    std::vector<KSeg> segs;
    std::vector<int> blk;
    int off = 0;
    // FP32 launches with fracture blocks and more 256-row tiles than two
    // resident workgroups per CU cover use the three-per-CU variant (its
    // grid cap is larger)
    G.pc = 0;
    long tiles = 0;
    for (int q : G.idx) {
        const fim_model* m = items[q].m;
        if (m->use_pc) G.pc = m->pc_dec ? 2 : 1;   // one mode per batch (batch_check)
        tiles += krylov_grid(m->nA, KB_MAXB);
    }
    G.wide = G.pc && g == 0 && tiles > lead->pc_grid;
    for (int q : G.idx) {
        SolveItem& it = items[q];
        fim_model* m = it.m;
        KSeg k;
        k.ls = lsys(m);
        k.kb = kbufs(m, g == 0);
        k.nA = m->nA;
        k.blk0 = off;
        k.nblk = krylov_grid(m->nA, m->use_pc ? (G.wide ? m->pc_grid_wide : m->pc_grid)
                                              : KB_MAXB);
        k.active = it.active ? 1 : 0;
        k.tol2 = it.tol2;
        k.bnorm2 = it.bnorm2;
        k.maxit = m->o.krylov_maxit;
        k.pad = 0;
        for (int b = 0; b < k.nblk; b++) blk.push_back((int)segs.size());
        off += k.nblk;
        segs.push_back(k);
    }
    G.nblk = off;
    if (segs.empty()) return fim_status(FIM_OK);
    fim_model* m = lead;
    KSeg* hs = t.hsegs + (size_t)g * t.cap;
    std::memcpy(hs, segs.data(), segs.size() * sizeof(KSeg));
    HIPX(hipMemcpyAsync(t.dsegs + (size_t)g * t.cap, hs, segs.size() * sizeof(KSeg),
                        hipMemcpyHostToDevice, s));
    if (segs.size() > 1) {   // one-model launches do not read the block map
        int* hb = t.hblk + (size_t)g * t.cap * KB_MAXB;
        std::memcpy(hb, blk.data(), blk.size() * sizeof(int));
        HIPX(hipMemcpyAsync(t.dblk + (size_t)g * t.cap * KB_MAXB, hb, blk.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
    }
    return FIM_OK;
}

static fim_status read_status(fim_model* lead, SolveTable& t, Group* G, std::vector<SolveItem>& items,
                              hipStream_t s, bool flush = true) {
    fim_model* m = lead;
    for (int g = 0; g < 2; g++)
        if (!G[g].idx.empty())
            launch_seg_status(t.dsegs + (size_t)g * t.cap, (int)G[g].idx.size(),
                              t.hstat_dev + (size_t)g * t.cap, s);
    HIPX(spin_sync(lead, s));
    if (flush) pflush(lead);
    (void)items;
    return FIM_OK;
}

// a launch over group g covers a single model
static bool solo_of(SolveTable& t, Group* G, int g) {
    (void)t;
    return G[g].idx.size() == 1;
}

static const SegStatus& status_of(SolveTable& t, Group* G, int g, int pos) {
    return t.hstat[(size_t)g * t.cap + pos];
}

// Local linear solves J_A x = -F_A of several models at once (one model:
// a batch of one), by iterative refinement around BiCGStab on the
// block-Jacobi scaled systems.  In mixed precision the inner solves run in
// FP32; a model whose pass fails to cut its FP64 residual norm by at least
// 10 % (stagnation or breakdown on a badly conditioned fracture subsystem)
// has the pass undone and continues with the FP64 Krylov.
// prepped: each model's block-Jacobi scaling (k_precond) and zero initial
// guess were already queued on its own stream (batched steps)
static void solve_prep(fim_model* m, hipStream_t s) {
    launch_precond(m->B, m->o.precision == FIM_MIXED, m->nA, lsys(m), m->dinv, m->At, s);
    launch_fill_f64(m->x64, (long)m->nA * m->B, 0.0, s);
}

// Relative tolerance of this Newton iteration's linear solve: lin_rtol, or,
// in full Newton and Algorithm 1, the inexact Newton forcing term of
// Eisenstat and Walker (1996, choice 2, gamma 0.9, alpha (1 + sqrt 5) / 2,
// with their safeguard) between lin_rtol and forcing_max, from the norms of the
// iterations' local residuals (the first iteration of a timestep takes
// forcing_max).  Algorithm 2's sweeps (phase 2, both forms) keep one such
// sequence per subdomain, over that subdomain's own solves; the
// residual-based mode starts its sequence at lin_rtol.  Algorithm 2's
// subdomain-building phase (the subdomains are built from the updates'
// magnitudes), tight mode and solves outside a Newton iteration
// (fim_inspect_solve) take lin_rtol.
// exponent of choice 2: the golden ratio, the order of the secant method
constexpr double EW_ALPHA = 1.6180339887498949;

static double forcing_eta(fim_model* m, double fnorm2) {
    const double lo = m->o.lin_rtol, hi = m->o.forcing_max;
    // (a subdomain workspace of the additive form solves for its owner)
    fim_model* o = m->is_clone ? m->ew_owner : m;
    const bool dd2 = o && (m->step_mode == FIM_DD || m->step_mode == FIM_DD_ADD) &&
                     o->dd_phase == 2 && m->dd_cur >= 0;
    if (!(hi > lo) || m->o.tight || !o || !o->in_step || (m->is_clone && !dd2) ||
        (m->step_mode != FIM_FULL && m->step_mode != FIM_LOCAL && m->step_mode != FIM_RESID &&
         !dd2))
        return lo;
    if (dd2 && (int)o->dd_ew_f.size() <= m->dd_cur) {
        o->dd_ew_f.resize(m->dd_cur + 1, 0.0);
        o->dd_ew_eta.resize(m->dd_cur + 1, 0.0);
    }
    double& fprev = dd2 ? o->dd_ew_f[m->dd_cur] : m->ew_fprev;
    double& eprev = dd2 ? o->dd_ew_eta[m->dd_cur] : m->ew_eta;
    const double fn = std::sqrt(fnorm2);
    // the first solve of the step (or of the subdomain); the residual-based
    // mode solves its first iteration, on every cell, to lin_rtol: its
    // error measure, which picks the next iterations' cells, needs it
    double eta = m->step_mode == FIM_RESID ? lo : hi;
    if (fprev > 0.0 && std::isfinite(fn)) {
        const double r = fn / fprev;
        eta = 0.9 * std::pow(r, EW_ALPHA);
        const double safe = 0.9 * std::pow(eprev, EW_ALPHA);
        if (safe > 0.1) eta = std::max(eta, safe);
    }
    eta = std::min(hi, std::max(lo, eta));
    fprev = fn;
    eprev = eta;
    return eta;
}

static fim_status solve_batch(std::vector<fim_model*>& ms, SolveTable& t, hipStream_t s,
                              bool prepped = false) {
    fim_model* lead = ms[0];
    fim_model* m = lead;
    const int K = (int)ms.size();
    std::vector<SolveItem> items(K);
    Group G[2];
    for (int q = 0; q < K; q++) {
        fim_model* mq = ms[q];
        SolveItem& it = items[q];
        it = SolveItem{mq, mq->o.precision == FIM_MIXED, false, true, 0, 0, 0, 0, 0, 0, 0, 0};
        if (!prepped) {
            const int pi = pbeg(lead, PK_PRECOND);
            launch_precond(mq->B, it.fp32, mq->nA, lsys(mq), mq->dinv, mq->At, s);
            pend(lead, pi, mq->nA);
        }
        if (mq->use_pc && K == 1) {
            const int pv = pbeg(lead, PK_PCINV);
            launch_pc_invert(mq->B, it.fp32, mq->pc_inv_grid, lsys(mq), mq->At, mq->pclist,
                             &mq->dint[6], mq->pcoff, mq->pcM, mq->pc_dec, s);
            pend(lead, pv, mq->nA);
        }
        if (!prepped) launch_fill_f64(mq->x64, (long)mq->nA * mq->B, 0.0, s);
        G[it.fp32 ? 0 : 1].idx.push_back(q);
    }
    if (K > 1) {
        // the fracture blocks of all members in one launch per precision
        // (each member's inversion alone is a few waves and latency-bound)
        for (int g = 0; g < 2; g++) {
            std::vector<PcSeg> pcs;
            for (int q : G[g].idx) {
                fim_model* mq = ms[q];
                if (mq->use_pc)
                    pcs.push_back(PcSeg{lsys(mq), mq->At, mq->pclist, &mq->dint[6], mq->pcoff,
                                        mq->pcM});
            }
            if (pcs.empty()) continue;
            PcSeg* dpc = t.dpc + (size_t)g * t.cap;
            int* dpref = t.dpref + (size_t)g * (t.cap + 1);
            HIPX(hipMemcpyAsync(dpc, pcs.data(), pcs.size() * sizeof(PcSeg),
                                hipMemcpyHostToDevice, s));
            const int pv = pbeg(lead, PK_PCINV);
            // one fracture-block mode per batch (batch_check)
            bool dec = false;
            for (int q : G[g].idx) dec = dec || (ms[q]->use_pc && ms[q]->pc_dec);
            launch_pc_invert_batch(lead->B, g == 0, (dec ? 20 : 8) * lead->cus, dpc,
                                   (int)pcs.size(), dpref, dec, s);
            pend(lead, pv, lead->nA);
        }
    }
    const int b = lead->B;
    for (int g = 0; g < 2; g++) TRY(upload_group(lead, t, g, G[g], items, s));
    int pi = pbeg(lead, PK_IR);
    for (int g = 0; g < 2; g++)
        launch_ir_residual(b, g == 0, solo_of(t, G, g), t.dsegs + (size_t)g * t.cap,
                           t.dblk + (size_t)g * t.cap * KB_MAXB, G[g].nblk, true, s);
    pend(lead, pi, lead->nA);
    if (lead->prof.on)
        HIPX(hipMemcpyAsync(&lead->hint[4], &lead->dint[4], 2 * sizeof(int), hipMemcpyDeviceToHost,
                            s));
    TRY(read_status(lead, t, G, items, s));
    if (lead->prof.on) {
        lead->cur_nnzb = lead->hint[4];
        // FP32 entries one application reads: (rows b)^2 per block, or
        // rows^2 b with the unknowns decoupled
        lead->cur_pcn2 = lead->use_pc ? (double)lead->hint[5] * lead->B *
                                            (lead->pc_dec ? 1 : lead->B)
                                      : 0.0;
    }
    for (int g = 0; g < 2; g++)
        for (size_t pos = 0; pos < G[g].idx.size(); pos++) {
            SolveItem& it = items[G[g].idx[pos]];
            const SegStatus& st = status_of(t, G, g, (int)pos);
            it.rir2 = st.rir2;
            it.bnorm2 = st.bnorm2;
            it.fnorm2 = st.rir2;
            const double eta = forcing_eta(it.m, it.fnorm2);
            it.target2 = eta * eta * it.fnorm2;
        }
    const int max_refine = lead->o.max_refine;
    const int check = lead->o.check_every;
    for (int pass = 0; pass < max_refine; pass++) {
        int nact = 0;
        for (SolveItem& it : items) {
            it.done_outer = !(it.rir2 > it.target2) || !std::isfinite(it.rir2);
            it.active = !it.done_outer;
            if (!it.active) continue;
            nact++;
            it.passes++;
            fim_model* mq = it.m;
            // inner target: the reduction this pass needs, not below what
            // the Krylov precision can deliver
            const double need = 0.5 * std::sqrt(it.target2 / it.rir2);
            const double floor_ = it.fp32 ? std::max(mq->o.inner_rtol, 1e-6) : 1e-15;
            const double inner = std::max(need, floor_);
            it.tol2 = inner * inner * it.bnorm2;
        }
        if (!nact) break;
        for (int g = 0; g < 2; g++) TRY(upload_group(lead, t, g, G[g], items, s));
        // ---- BiCGStab in lockstep; finished models return at once.  The
        // next block of iterations is queued before the status of the
        // current one is examined, so the GPU does not idle during the
        // host check (without profiling, whose records need the stream
        // drained).
        const bool ahead = !lead->prof.on;
        // a block of len iterations; its last kernel S writes every model's
        // Krylov status into slot sl (2 slots) of the pinned status table
        auto queue_chunk = [&](int first_it, int len, int sl) {
            for (int c = 0; c < len; c++)
                for (int w = 0; w < 2; w++)
                    for (int g = 0; g < 2; g++) {
                        if (!G[g].nblk) continue;
                        const int q = pbeg_ext(lead, PK_BICG_A + w, c);
                        SegStatus* rec = (w == 1 && c == len - 1)
                                             ? t.hstat_dev + (size_t)(2 + 2 * sl + g) * t.cap
                                             : nullptr;
                        launch_bicg_part(w, b, g == 0, solo_of(t, G, g), G[g].pc,
                                         t.dsegs + (size_t)g * t.cap,
                                         t.dblk + (size_t)g * t.cap * KB_MAXB, G[g].nblk,
                                         first_it + c, s, q >= 0 ? lead->prof.pend[q].a : nullptr,
                                         q >= 0 ? lead->prof.pend[q].b : nullptr, rec, G[g].wide);
                        if (q >= 0) lead->prof.pend[q].rows = lead->nA;
                    }
        };
        // the event that tells the host slot sl is written
        auto queue_status = [&](int sl) -> fim_status {
            HIPX(hipEventRecord(t.ev[sl], s));
            return FIM_OK;
        };
        // Iterations queued so far, and the length of the next block: near
        // convergence the block shrinks to what the observed residual
        // decay predicts (plus a margin), and none is queued while the
        // work in flight is predicted to suffice, so that few launches run
        // after the solve has finished.  Blocks are never shorter than 2.
        int queued = 0;
        int next_len = check;
        auto plan_next = [&](int sl) {
            double need = -1e30;   // iterations still to queue, over the models
            bool unknown = false;
            for (int g = 0; g < 2; g++)
                for (size_t pos = 0; pos < G[g].idx.size(); pos++) {
                    const int q = G[g].idx[pos];
                    if (!items[q].active) continue;
                    const SegStatus& st = t.hstat[(size_t)(2 + 2 * sl + g) * t.cap + pos];
                    if (st.done) continue;
                    const double rr = st.rr, tol2 = items[q].tol2, r0 = items[q].bnorm2;
                    // average decay per iteration since the start of the pass
                    // (x0 = 0, so |r_0|^2 = |b~|^2): BiCGStab residuals are
                    // too erratic from one check to the next
                    if (st.iters > 0 && rr > 0.0 && r0 > 0.0 && tol2 > 0.0) {
                        const double rate = std::pow(rr / r0, 1.0 / st.iters);
                        if (rate < 0.999) {
                            const double rem = std::log(tol2 / rr) / std::log(rate);
                            need = std::max(need, rem - (queued - st.iters));
                        } else {
                            unknown = true;
                        }
                    } else {
                        unknown = true;
                    }
                }
            // nothing more while the queued work is predicted to finish the
            // solve with an iteration to spare: launches queued past
            // convergence return at once but still cost a dispatch each
            next_len = unknown ? check
                       : need <= -1.0 ? 0
                                      : std::max(2, std::min(check, (int)std::ceil(need) + 2));
        };
        int before = 0;
        const int max_chunks = lead->o.krylov_maxit + 4;   // blocks are >= 1 iteration
        const int max_queued = lead->o.krylov_maxit + 2 * check;
        // blocks whose status is queued and not yet read (their slots, in
        // order; at most two, in alternating slots)
        int inflight[2] = {0, 0}, npend = 0, slot_next = 0;
        auto issue = [&](int len) -> fim_status {
            queue_chunk(queued, len, slot_next);
            queued += len;
            TRY(queue_status(slot_next));
            inflight[npend++] = slot_next;
            slot_next ^= 1;
            return FIM_OK;
        };
        TRY(issue(check));
        for (int chunk = 0; chunk < max_chunks; chunk++) {
            const bool more = queued < max_queued;
            if (more && (npend == 0 || (ahead && npend < 2 && next_len > 0)))
                TRY(issue(npend == 0 ? std::max(2, next_len) : next_len));
            if (npend == 0) break;   // (not reached: the cap ends the loop below)
            const int sl = inflight[0];
            inflight[0] = inflight[1];
            npend--;
            HIPX(spin_event(t.ev[sl]));
            // the lead model's iteration count tells which of its profiled
            // launches did work (later ones returned at once)
            for (int g = 0; g < 2; g++)
                for (size_t pos = 0; pos < G[g].idx.size(); pos++)
                    if (G[g].idx[pos] == 0 && lead->prof.on) {
                        const int its = t.hstat[(size_t)(2 + 2 * sl + g) * t.cap + pos].iters;
                        pflush(lead, its - before);
                        before = its;
                    }
            bool all = true;
            for (int g = 0; g < 2; g++)
                for (size_t pos = 0; pos < G[g].idx.size(); pos++)
                    if (items[G[g].idx[pos]].active &&
                        !t.hstat[(size_t)(2 + 2 * sl + g) * t.cap + pos].done)
                        all = false;
            if (all || (!more && npend == 0)) {
                // final iteration counts.  Without more work queued, the
                // status just read covers everything queued, and the
                // iteration cap has stopped every model inside it.
                for (int g = 0; g < 2; g++)
                    for (size_t pos = 0; pos < G[g].idx.size(); pos++)
                        t.hstat[(size_t)g * t.cap + pos] = t.hstat[(size_t)(2 + 2 * sl + g) * t.cap + pos];
                break;
            }
            if (ahead) plan_next(sl);
        }
        for (int g = 0; g < 2; g++)
            for (size_t pos = 0; pos < G[g].idx.size(); pos++) {
                SolveItem& it = items[G[g].idx[pos]];
                if (it.active) it.kry += status_of(t, G, g, (int)pos).iters;
            }
        pi = pbeg(lead, PK_IR);
        for (int g = 0; g < 2; g++) {
            launch_ir_accumulate(b, g == 0, solo_of(t, G, g), t.dsegs + (size_t)g * t.cap,
                                 t.dblk + (size_t)g * t.cap * KB_MAXB, G[g].nblk, s);
            launch_ir_residual(b, g == 0, solo_of(t, G, g), t.dsegs + (size_t)g * t.cap,
                               t.dblk + (size_t)g * t.cap * KB_MAXB, G[g].nblk, false, s);
        }
        pend(lead, pi, lead->nA);
        TRY(read_status(lead, t, G, items, s));
        // new residuals; FP32 passes that stalled are undone -> FP64
        bool moved = false;
        std::vector<int> keep32;
        for (size_t pos = 0; pos < G[0].idx.size(); pos++) {
            const int q = G[0].idx[pos];
            SolveItem& it = items[q];
            const SegStatus& st = status_of(t, G, 0, (int)pos);
            if (it.active && !(st.rir2 < 0.81 * it.rir2)) {
                fim_model* mq = it.m;
                launch_copy_f64(mq->x64, mq->xprev, (long)mq->nA * mq->B, s);
                launch_precond(mq->B, false, mq->nA, lsys(mq), mq->dinv, mq->At, s);
                it.fp32 = false;
                it.fallback = 1;
                G[1].idx.push_back(q);
                moved = true;
            } else {
                keep32.push_back(q);
                if (it.active) {
                    it.rir2 = st.rir2;
                    it.bnorm2 = st.bnorm2;
                }
            }
        }
        for (size_t pos = 0; pos < G[1].idx.size(); pos++) {
            SolveItem& it = items[G[1].idx[pos]];
            if (it.active && it.fallback != 1) {   // not moved in this pass
                const SegStatus& st = status_of(t, G, 1, (int)pos);
                it.rir2 = st.rir2;
                it.bnorm2 = st.bnorm2;
            }
        }
        if (moved) {
            // recompute the FP64 refinement residual of the moved models
            G[0].idx = keep32;
            for (SolveItem& it : items) it.active = it.fallback == 1 && !it.fp32 && it.active;
            for (int g = 0; g < 2; g++) TRY(upload_group(lead, t, g, G[g], items, s));
            launch_ir_residual(b, false, solo_of(t, G, 1), t.dsegs + (size_t)t.cap,
                               t.dblk + (size_t)t.cap * KB_MAXB, G[1].nblk, false, s);
            TRY(read_status(lead, t, G, items, s));
            for (size_t pos = 0; pos < G[1].idx.size(); pos++) {
                SolveItem& it = items[G[1].idx[pos]];
                if (it.active) {
                    const SegStatus& st = status_of(t, G, 1, (int)pos);
                    it.rir2 = st.rir2;
                    it.bnorm2 = st.bnorm2;
                }
                it.fallback = it.fallback ? 2 : 0;
            }
        }
    }
    for (SolveItem& it : items) {
        fim_model* mq = it.m;
        mq->last_kry = it.kry;
        mq->last_refine = it.passes;
        mq->last_fallback = it.fallback ? 1 : 0;
        mq->last_relres = it.fnorm2 > 0 ? std::sqrt(it.rir2 / it.fnorm2) : 0.0;
    }
    return FIM_OK;
}

static fim_status linear_solve(fim_model* m) {
    std::vector<fim_model*> one{m};
    if (m->noalloc) return solve_batch(one, m->nat, m->s);
    if (!m->solo.cap) TRY(table_alloc(m, m->solo, 1));
    return solve_batch(one, m->solo, m->s);
}

static bool converged(const fim_model* m, const NStat& ns) {
    bool ok = ns.dp_max < m->o.eps_conv;
    if (m->o.tight) ok = ok && ns.ds_max < m->o.eps_s && ns.nswitch == 0;
    return ok;
}

// Assembly + solve + update on the current active rows.
// Assembly of the current active rows (launch only).
static void newton_assemble(fim_model* m) {
    const int pi = pbeg(m, PK_ASSEMBLE);
    launch_assemble(m->fk, m->nA, lsys(m), m->g, m->f, m->u, m->st, m->Mn, 1.0 / m->step_dt, m->s);
    pend(m, pi, m->nA);
}

// the bookkeeping of the solve (no launch)
static void newton_update_stats(fim_model* m, fim_iter_stats* it) {
    if (it) {
        it->n_active = m->nA;
        it->krylov_iters = m->last_kry;
        it->refine_passes = m->last_refine;
        it->fp64_fallback = m->last_fallback;
        it->lin_relres = m->last_relres;
    }
    m->sum_active += m->nA;
    m->max_active = std::max(m->max_active, m->nA);
    m->step_kry += m->last_kry;
}

// the cell classes of the iteration (fim_flags_enable)
static void newton_classes(fim_model* m) {
    if (m->flags_on) {
        launch_fill_u8(m->classes, m->n, 0, m->s);
        launch_cell_classes(m->nA, m->l2g, m->bnd,
                            m->step_mode == FIM_LOCAL || m->step_mode == FIM_DD ||
                                m->step_mode == FIM_DD_ADD,
                            m->dp_abs,
                            m->o.eps_loc, m->classes, m->s);
    }
}

// Update after the solve (launch only) and the bookkeeping of the solve.
static void newton_update(fim_model* m, fim_iter_stats* it) {
    const int pi = pbeg(m, PK_UPDATE);
    launch_update(m->fk, m->nA, m->l2g, m->x64, m->u, m->st, m->n, m->f, m->o.ds_max,
                  m->dp_abs, m->part, m->ns, m->s);
    pend(m, pi, m->nA);
    newton_classes(m);
    newton_update_stats(m, it);
}

// Assembly + solve + update on the current active rows.
static fim_status local_newton(fim_model* m, fim_iter_stats* it) {
    newton_assemble(m);
    TRY(linear_solve(m));
    newton_update(m, it);
    return FIM_OK;
}

static fim_status prepare_active(fim_model* m, bool need_bnd) {
    compact(m);
    TRY(read_int(m));
    m->nA = m->hint[1];
    TRY(structure(m));
    if (need_bnd) {
        launch_fill_i32(&m->dint[2], 1, 0, m->s);
        launch_boundary(m->nA, m->l2g, m->g2l, m->g, m->bnd, &m->dint[2], m->s);
    }
    return FIM_OK;
}

// Localized fracture cells: close the active flags under fracture
// components (Algorithm 1 only; a no-op without localized fracture cells).
static void frac_closure(fim_model* m) {
    if (m->fclose)
        launch_frac_closure(m->nfcell, m->fcells, m->fcomp, m->ncomp, m->ftouch, m->act, m->s);
}

// The launches that start a timestep.  *pending: the step's first active
// set is compacted and its n_A (dint[1], copied to hint[1]) must be read
// before the structure pass (begin_finish); else n_A = n already.
// Host side of a timestep start.  Returns how the step's first active set
// is formed: 1 = the previous step's support, 2 = the always-active cells
// and their neighbour layers, 3 = all cells, 4 = all cells, already
// compacted (full Newton and the residual-based mode on a ready set).
static int begin_state(fim_model* m, double dt, int mode) {
    m->ew_fprev = 0.0;
    m->ew_eta = 0.0;
    m->in_step = true;
    m->step_dt = dt;
    m->step_mode = mode;
    m->nu = 0;
    m->is_expand = true;
    m->sum_active = 0.0;
    m->max_active = 0;
    m->step_kry = 0;
    m->inspect_ready = false;
    if (mode == FIM_FULL || mode == FIM_RESID) {
        m->nA = m->n;
        return m->full_ready ? 4 : 3;
    }
    return m->have_history ? 1 : 2;
}

static fim_status begin_launch(fim_model* m, double dt, int mode, bool* pending) {
    *pending = false;
    const int pi = pbeg(m, PK_SETUP);
    launch_copy_state(m->B, m->n, m->u, m->st, m->un, m->stn, m->s);
    launch_accumulation(m->fk, m->n, m->un, m->stn, m->g, m->f, m->Mn, m->s);
    pend(m, pi, m->n);
    (void)begin_state(m, dt, mode);
    if (mode == FIM_FULL || mode == FIM_RESID) {
        // the residual-based localization starts every step on all cells
        if (!m->full_ready) {
            launch_fill_u8(m->act, m->n, 1, m->s);
            compact(m);
            launch_status_out(nullptr, m->dint, nullptr, m->hint_dev, m->s);
            *pending = true;
        }
        m->nA = m->n;
        return FIM_OK;
    }
    m->full_ready = false;
    const bool dd = mode == FIM_DD || mode == FIM_DD_ADD;
    const int layers = dd ? m->o.m_layers_dd : m->o.m_layers;
    if (m->have_history) {
        HIPX(hipMemcpyAsync(m->act, m->supp, m->n, hipMemcpyDeviceToDevice, m->s));
    } else {
        launch_fill_u8(m->act, m->n, 0, m->s);
        launch_mark_seeds(m->n, m->g, layers, m->act, m->lvl, m->s);
    }
    if (mode == FIM_LOCAL) frac_closure(m);
    if (mode == FIM_DD_ADD) {
        if (!m->dd_owner) TRY(dal(m, &m->dd_owner, (size_t)m->n));
        launch_fill_i32(m->dd_owner, m->n, -1, m->s);
    }
    if (dd) {
        launch_fill_f64(m->last_dp, m->n, 0.0, m->s);
        HIPX(hipMemcpyAsync(m->vt, m->act, m->n, hipMemcpyDeviceToDevice, m->s));
        m->subs.clear();
        m->dd_ew_f.clear();
        m->dd_ew_eta.clear();
        m->sd_used = m->ob_used = 0;
        m->dd_phase = 1;
        m->dd_valid = true;
        m->dd_sweeps = 0;
        m->dd_next = 0;
        m->dd_k = 0;
    }
    compact(m);
    launch_status_out(nullptr, m->dint, nullptr, m->hint_dev, m->s);
    *pending = true;
    return FIM_OK;
}

// After the compaction of begin_launch has been read (hint[1]): the
// structure of the first local system, V_B and Algorithm 2's outer layer.
static fim_status begin_finish(fim_model* m) {
    const int mode = m->step_mode;
    if (mode == FIM_FULL || mode == FIM_RESID) {
        m->nA = m->hint[1];
        TRY(structure(m));
        m->full_ready = true;
        m->nA = m->n;
        return FIM_OK;
    }
    m->nA = m->hint[1];
    TRY(structure(m));
    launch_fill_i32(&m->dint[2], 1, 0, m->s);
    launch_boundary(m->nA, m->l2g, m->g2l, m->g, m->bnd, &m->dint[2], m->s);
    if (mode == FIM_DD || mode == FIM_DD_ADD) {
        launch_fill_u8(m->outer, m->n, 0, m->s);
        launch_outer_layer(m->nA, m->l2g, m->act, m->g, m->outer, m->s);
    }
    return FIM_OK;
}

static fim_status begin_step(fim_model* m, double dt, int mode) {
    bool pending = false;
    TRY(begin_launch(m, dt, mode, &pending));
    if (!pending) return FIM_OK;
    HIPX(spin_sync(m, m->s));
    pflush(m);
    return begin_finish(m);
}

static void commit(fim_model* m) {
    launch_support(m->n, m->u, m->un, m->o.eps_loc, m->g, m->supp, m->s);
    m->have_history = true;
    m->in_step = false;
}

static fim_status rollback(fim_model* m) {
    launch_copy_state(m->B, m->n, m->un, m->stn, m->u, m->st, m->s);
    m->in_step = false;
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

// ------------------------------------------------------- Algorithm 2 util
static fim_status dd_grow(fim_model* m, int** buf, long* cap, long need) {
    if (need <= *cap) return FIM_OK;
    long nc = std::max(need, 2 * *cap);
    int* nb = nullptr;
    TRY(dal(m, &nb, nc));
    if (*buf) {
        HIPX(hipMemcpyAsync(nb, *buf, *cap * sizeof(int), hipMemcpyDeviceToDevice, m->s));
        HIPX(hipStreamSynchronize(m->s));
        HIPX(hipFree(*buf));
    }
    *buf = nb;
    *cap = nc;
    return FIM_OK;
}

// store V_A^k (= current l2g) and its outer layer (flags in m->outer)
static fim_status dd_store(fim_model* m) {
    if ((int)m->subs.size() >= MAX_SUBS) {
        m->err = "Algorithm 2 built more than 64 subdomains";
        return FIM_NOT_CONVERGED;
    }
    DDSub sd;
    TRY(dd_grow(m, &m->sd_cells, &m->sd_cap, m->sd_used + m->nA));
    HIPX(hipMemcpyAsync(m->sd_cells + m->sd_used, m->l2g, (size_t)m->nA * sizeof(int),
                        hipMemcpyDeviceToDevice, m->s));
    sd.cells_off = m->sd_used;
    sd.cells_n = m->nA;
    m->sd_used += m->nA;
    // compact the outer-layer flags into a list, using the upper halves of
    // the l2g / g2l buffers as scratch
    launch_compact(m->outer, m->n, m->blk, m->l2g + m->n, m->g2l + m->n, &m->dint[3], m->s);
    TRY(read_int(m));
    const int nob = m->hint[3];
    TRY(dd_grow(m, &m->sd_outer, &m->ob_cap, m->ob_used + nob + 1));
    HIPX(hipMemcpyAsync(m->sd_outer + m->ob_used, m->l2g + m->n, (size_t)nob * sizeof(int),
                        hipMemcpyDeviceToDevice, m->s));
    sd.outer_off = m->ob_used;
    sd.outer_n = nob;
    m->ob_used += nob;
    m->subs.push_back(sd);
    return FIM_OK;
}

// activate a stored subdomain: l2g = its list, g2l = inverse
static fim_status dd_activate(fim_model* m, int k) {
    const DDSub& sd = m->subs[k];
    launch_fill_u8(m->act, m->n, 0, m->s);
    launch_scatter_flags(sd.cells_n, m->sd_cells + sd.cells_off, m->act, m->s);
    compact(m);
    m->nA = sd.cells_n;
    TRY(structure(m));
    return FIM_OK;
}

// ------------------------------------------- additive Algorithm 2 workspaces
// A subdomain workspace: shares the parent's static data, state and options
// (pointers copied), owns the buffers of one local system (active flags,
// compaction, matrix, right-hand side, Krylov vectors and scalars,
// fracture-block layout and inverses, the update's |dp| and partials).
static void free_clone(fim_model* c) {
    void* own[] = {c->act, c->l2g, c->g2l, c->swidth, c->blk, c->col, c->J, c->F, c->dinv,
                   c->At, c->x64, c->rir, c->part, c->kvec, c->xprev, c->sc, c->part_ir,
                   c->ns, c->dint, c->dp_abs, c->pcinfo, c->pcoff, c->pcM, c->pclist};
    for (void* p : own)
        if (p) (void)hipFree(p);
    if (c->hsc) (void)hipHostFree(c->hsc);
    if (c->hns) (void)hipHostFree(c->hns);
    if (c->hint) (void)hipHostFree(c->hint);
    if (c->hpart) (void)hipHostFree(c->hpart);
    if (c->sync_ev) (void)hipEventDestroy(c->sync_ev);
    delete c;
}

static fim_status make_clone(fim_model* m, fim_model** out) {
    fim_model* c = new fim_model();
    c->is_clone = true;
    c->n = m->n; c->nconn = m->nconn; c->B = m->B; c->fk = m->fk;
    c->o = m->o; c->f = m->f; c->s = m->s; c->g = m->g;
    c->adj_ptr = m->adj_ptr; c->adj_nbr = m->adj_nbr; c->adj_T = m->adj_T;
    c->pv = m->pv; c->depth = m->depth; c->wi = m->wi; c->bhp = m->bhp; c->flags = m->flags;
    c->max_deg = m->max_deg; c->slot_cap = m->slot_cap;
    c->u = m->u; c->un = m->un; c->Mn = m->Mn; c->st = m->st; c->stn = m->stn;
    c->use_pc = m->use_pc; c->pc_cap = m->pc_cap; c->pc_grid = m->pc_grid;
    c->pc_dec = m->pc_dec;
    c->funit = m->funit;
    c->pc_grid_wide = m->pc_grid_wide; c->pc_inv_grid = m->pc_inv_grid; c->pc_nfc = m->pc_nfc;
    c->frac_id = m->frac_id; c->ford = m->ford; c->cus = m->cus; c->dev = m->dev;
    const size_t nn = (size_t)m->n, B = (size_t)m->B;
    const size_t nsl = (nn + SLICE - 1) / SLICE;
    const size_t ntile = std::max((nn + TILE - 1) / TILE, (nsl + TILE - 1) / TILE) + 1;
    fim_status r = FIM_OK;
    auto al = [&](auto** p, size_t cnt) {
        if (r == FIM_OK) r = dal(c, p, cnt);
    };
    al(&c->act, nn);
    al(&c->l2g, 2 * nn);
    al(&c->g2l, 2 * nn);
    al(&c->swidth, nsl + 1);
    al(&c->blk, ntile);
    al(&c->col, (size_t)c->slot_cap);
    al(&c->J, (size_t)c->slot_cap * B * B);
    al(&c->F, nn * B);
    al(&c->dinv, nn * B * B);
    if (r == FIM_OK) r = dalloc(c, &c->At, (size_t)c->slot_cap * B * B * sizeof(double));
    al(&c->x64, nn * B);
    al(&c->rir, nn * B);
    al(&c->part, 4 * ((nn * B + NT - 1) / NT + 1));
    if (r == FIM_OK) r = dalloc(c, &c->kvec, 9 * nn * B * sizeof(double));
    al(&c->xprev, nn * B);
    al(&c->sc, 1);
    al(&c->part_ir, 14 * KB_MAXB);
    al(&c->ns, 1);
    al(&c->dint, 8);
    al(&c->dp_abs, nn);
    if (c->use_pc) {
        al(&c->pcinfo, nn);
        al(&c->pcoff, nn);
        al(&c->pcM, (size_t)c->pc_nfc * pc_cell_stride(m->B));
        al(&c->pclist, 2 * ((size_t)c->pc_nfc / 2 + 1));
    }
    if (r == FIM_OK &&
        (hipHostMalloc((void**)&c->hsc, sizeof(KScal)) != hipSuccess ||
         hipHostMalloc((void**)&c->hns, sizeof(NStat)) != hipSuccess ||
         hipHostMalloc((void**)&c->hint, 8 * sizeof(int)) != hipSuccess ||
         hipHostMalloc((void**)&c->hpart, 2 * KB_MAXB * sizeof(double)) != hipSuccess ||
         hipEventCreateWithFlags(&c->sync_ev, hipEventDisableTiming) != hipSuccess))
        r = FIM_E_NOMEM;
    if (r != FIM_OK) {
        m->err = "subdomain workspace: " + (c->err.empty() ? std::string("allocation failed") : c->err);
        free_clone(c);
        return r;
    }
    m->bytes += c->bytes;
    *out = c;
    return FIM_OK;
}

// Phase-1 set logic of Algorithm 2 (Section 4.4, Step 1) after the solve
// on V_A^k (l2g, n_A), with the boundary flags of V_B^k in bnd and the
// update in dp_abs: the layers-layer neighbourhoods of the cells of V_B^k
// with |dp| >= eps join V_T and form V_A^{k+1}.  When there are any,
// V_A^{k+1} becomes the active set (compacted), V_B^{k+1} =
// boundary(V_T) ^ V_A^{k+1} goes into bnd and the outer layer dB^{k+1}
// into outer.  *expand receives whether any cell qualified (host read).
static fim_status dd_expand_sets(fim_model* m, double eps, int layers, bool* expand) {
    launch_fill_u8(m->act2, m->n, 0, m->s);
    launch_fill_i32(m->dint, 1, 0, m->s);
    launch_mark_expand(m->nA, m->l2g, m->bnd, m->dp_abs, eps, layers, m->g, m->vt, m->act2,
                       m->dint, m->lvl, m->s);
    TRY(read_int(m));
    *expand = m->hint[0] != 0;
    if (*expand) {
        HIPX(hipMemcpyAsync(m->act, m->act2, m->n, hipMemcpyDeviceToDevice, m->s));
        TRY(prepare_active(m, false));
        launch_dd_boundary(m->nA, m->l2g, m->vt, m->g, m->bnd, m->s);
        launch_fill_u8(m->outer, m->n, 0, m->s);
        launch_outer_layer(m->nA, m->l2g, m->act, m->g, m->outer, m->s);
    }
    return FIM_OK;
}

// Phase 2 of Algorithm 2 (Section 4.4, Step 2): the next subdomain in
// sweep order whose largest latest update over V_A^k and its outer layer
// dB^k (smax[k]) is at least eps.  The search starts at position next in
// [0, N] (one past the subdomain solved last; N when that was the last of
// the list) and runs cyclically; -1 when no subdomain qualifies.
// *new_sweep: the search passed the end of the list, so the pick opens
// the next sweep.
static int dd_pick(const double* smax, int N, double eps, int next, bool* new_sweep) {
    *new_sweep = false;
    for (int q = 0; q < N; q++) {
        const int pos = next + q;
        const int k = pos % N;
        if (smax[k] >= eps) {
            *new_sweep = pos >= N;
            return k;
        }
    }
    return -1;
}

// ----------------------------------------------------------- C ABI
extern "C" {

void fim_default_options(fim_options* o) {
    const double psi = 6894.757293168;
    std::memset(o, 0, sizeof(*o));
    o->eps_conv = 0.3 * psi;
    o->eps_loc = 0.3 * psi;
    o->eps_s = 1e-10;
    o->tight = 0;
    o->m_layers = 2;
    o->m_layers_dd = 4;
    o->max_newton = 25;
    o->max_sweeps = 40;
    o->auto_cut = 0;
    o->max_cuts = 8;
    o->ds_max = 0.2;
    o->precision = FIM_FP64;
    o->lin_rtol = 1e-4;
    o->inner_rtol = 1e-5;
    o->krylov_maxit = 2000;
    o->max_refine = 20;
    o->check_every = 4;
    o->precond = FIM_PC_FRACTURE;
    o->eps_res = 1e-6;
    o->res_layers = 1;
    o->forcing_max = 0.1;
}

static thread_local std::string g_create_err;

const char* fim_last_error(const fim_model* m) { return m ? m->err.c_str() : g_create_err.c_str(); }
int32_t fim_num_cells(const fim_model* m) { return m ? m->n : 0; }
int32_t fim_block_size(const fim_model* m) { return m ? m->B : 0; }

static void free_all(fim_model* m) {
    table_free(m->solo);
    // the device parts of the allocation-free table are the scratch array
    m->nat.dsegs = nullptr;
    m->nat.dblk = nullptr;
    table_free(m->nat);
    for (const ProfRec& r : m->prof.pend) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : m->prof.pool) (void)hipEventDestroy(e);
    void* ptrs[] = {m->adj_ptr, m->adj_nbr, m->adj_T, m->pv, m->depth, m->wi, m->bhp, m->flags,
                    m->u, m->un, m->Mn, m->dp_abs, m->last_dp, m->st, m->stn, m->act, m->act2,
                    m->supp, m->bnd, m->vt, m->outer, m->l2g, m->g2l, m->swidth,
                    m->blk, m->col, m->J, m->F, m->dinv, m->At, m->x64, m->xprev, m->rir, m->part,
                    m->kvec, m->sc, m->ns, m->dint, m->dsub, m->sd_cells, m->sd_outer,
                    m->part_ir, m->classes, m->frac_id, m->ford, m->funit, m->pcinfo, m->pcoff,
                    m->pcM, m->pclist, m->lvl, m->usave, m->stsave, m->suppsave,
                    m->fcells, m->fcomp, m->ftouch, m->dd_owner};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (m->hsc) (void)hipHostFree(m->hsc);
    if (m->hns) (void)hipHostFree(m->hns);
    if (m->hint) (void)hipHostFree(m->hint);
    if (m->hsub) (void)hipHostFree(m->hsub);
    if (m->hpart) (void)hipHostFree(m->hpart);
    if (m->sync_ev) (void)hipEventDestroy(m->sync_ev);
    if (m->own_stream && m->s) (void)hipStreamDestroy(m->s);
}

static fim_status validate(const fim_model_desc* d, std::string& e) {
    if (!d) { e = "null description"; return FIM_E_ARG; }
    const int n = d->n_cells;
    if (n <= 0) { e = "n_cells must be positive"; return FIM_E_ARG; }
    if (d->n_conn < 0 || d->n_perf < 0) { e = "negative count"; return FIM_E_ARG; }
    if (!d->pv_ref || !d->depth || (d->n_conn && (!d->conn_i || !d->conn_j || !d->conn_T)) ||
        (d->n_perf && (!d->perf_cell || !d->perf_wi || !d->perf_bhp))) {
        e = "null array";
        return FIM_E_ARG;
    }
    const int k = d->fluid.kind;
    if (k < 1 || k > 3) { e = "fluid kind must be 1, 2 or 3"; return FIM_E_ARG; }
    for (int i = 0; i < n; i++) {
        if (!(d->pv_ref[i] > 0.0) || !std::isfinite(d->pv_ref[i])) {
            e = "pore volume must be positive at cell " + std::to_string(i);
            return FIM_E_ARG;
        }
        if (!std::isfinite(d->depth[i])) { e = "non-finite depth"; return FIM_E_ARG; }
    }
    for (int c = 0; c < d->n_conn; c++) {
        const int a = d->conn_i[c], b = d->conn_j[c];
        if (a < 0 || b >= n || a >= b) {
            e = "connection " + std::to_string(c) + " needs 0 <= conn_i < conn_j < n";
            return FIM_E_ARG;
        }
        if (!(d->conn_T[c] >= 0.0) || !std::isfinite(d->conn_T[c])) {
            e = "transmissibility must be finite and >= 0";
            return FIM_E_ARG;
        }
    }
    if (d->frac_id)
        for (int i = 0; i < n; i++)
            if (d->frac_id[i] < -1) { e = "frac_id must be >= -1"; return FIM_E_ARG; }
    std::vector<uint8_t> seen(n, 0);
    for (int p = 0; p < d->n_perf; p++) {
        const int c = d->perf_cell[p];
        if (c < 0 || c >= n) { e = "perforation cell out of range"; return FIM_E_ARG; }
        if (seen[c]) { e = "at most one perforation per cell"; return FIM_E_ARG; }
        seen[c] = 1;
        if (!(d->perf_wi[p] >= 0.0) || !std::isfinite(d->perf_bhp[p])) {
            e = "invalid well index or BHP";
            return FIM_E_ARG;
        }
    }
    return FIM_OK;
}

// Units of the fracture blocks.  Per fracture, its cells in index order
// (position p); u = the largest position distance of a connection between
// two of its cells when that is at most cap (a layered fracture numbered
// segment by segment: u = its layers, one unit = one segment's cells over
// the layers), else 1.  funit[i] = (p / u) << 8 | cap / u for a fracture
// cell (a block holds at most cap / u whole units, so at most cap cells).
// False if a fracture has more units than the 23 bits of the unit field.
static bool fracture_units(int n, const int* frac_id, const std::vector<int>& deg,
                           const std::vector<int>& nbr, int cap, std::vector<int>& funit) {
    std::vector<std::pair<int, int>> fc;   // (fracture, cell), cells ascending
    for (int i = 0; i < n; i++)
        if (frac_id[i] >= 0) fc.emplace_back(frac_id[i], i);
    std::stable_sort(fc.begin(), fc.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                         return a.first < b.first;
                     });
    std::vector<int> pos(n, 0);
    funit.assign(n, 0);
    for (size_t a = 0; a < fc.size();) {
        size_t e = a;
        while (e < fc.size() && fc[e].first == fc[a].first) e++;
        for (size_t q = a; q < e; q++) pos[fc[q].second] = (int)(q - a);
        int bw = 0;
        for (size_t q = a; q < e; q++) {
            const int i = fc[q].second;
            for (int k = deg[i]; k < deg[i + 1]; k++) {
                const int j = nbr[k];
                if (frac_id[j] == fc[a].first) bw = std::max(bw, std::abs(pos[j] - pos[i]));
            }
        }
        const int u = (bw >= 1 && bw <= cap) ? bw : 1;
        if ((e - a - 1) / u >= ((size_t)1 << 23)) return false;
        for (size_t q = a; q < e; q++)
            funit[fc[q].second] = ((int)(q - a) / u) << 8 | std::min(255, cap / u);
        a = e;
    }
    return true;
}

fim_status fim_create_model(const fim_model_desc* d, const fim_options* o,
                            void* hip_stream, fim_model** out) {
    if (!out) return FIM_E_ARG;
    *out = nullptr;
    std::string e;
    fim_status vs = validate(d, e);
    if (vs != FIM_OK) {
        g_create_err = e;
        return vs;
    }
    fim_model* m = new fim_model();
    if (o) m->o = *o;
    else fim_default_options(&m->o);
    if (m->o.check_every <= 0) m->o.check_every = 8;
    {
        // the fused fracture-block product kernels keep two workgroups per
        // CU resident; more tiles than that are looped over inside them
        // rather than launched as a second round of workgroups
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0) {
            m->pc_grid = std::min(KB_MAXB, 2 * cus);
            m->pc_grid_wide = std::min(KB_MAXB, 3 * cus);
            m->cus = cus;
        }
        m->dev = dev;
    }
    if (m->o.m_layers < 0 || m->o.m_layers > MAX_LAYERS || m->o.m_layers_dd < 0 ||
        m->o.m_layers_dd > MAX_LAYERS || m->o.res_layers < 0 ||
        m->o.res_layers > MAX_LAYERS) {
        g_create_err = "neighbour layers must be in [0, 8]";
        delete m;
        return FIM_E_ARG;
    }
    if (!(m->o.eps_res >= 0.0) || !std::isfinite(m->o.eps_res)) {
        g_create_err = "eps_res must be finite and >= 0";
        delete m;
        return FIM_E_ARG;
    }
    if (!(m->o.forcing_max >= 0.0) || !std::isfinite(m->o.forcing_max)) {
        g_create_err = "forcing_max must be finite and >= 0";
        delete m;
        return FIM_E_ARG;
    }
    if (m->o.precond != FIM_PC_JACOBI && m->o.precond != FIM_PC_FRACTURE &&
        m->o.precond != FIM_PC_FRACTURE_COUPLED) {
        g_create_err = "unknown preconditioner";
        delete m;
        return FIM_E_ARG;
    }
    const int n = d->n_cells;
    m->n = n;
    m->nconn = d->n_conn;
    m->fk = d->fluid.kind;
    m->B = m->fk;
    const fim_fluid& ff = d->fluid;
    m->f = DevFluid{ff.kind, ff.p_ref, ff.rho_ref, ff.c, ff.mu, ff.rho_w, ff.c_w, ff.mu_w,
                    ff.rho_o, ff.c_o, ff.mu_o, ff.swc, ff.sor, ff.rs_b, ff.p_b, ff.bo_slope,
                    ff.bg_c, ff.rho_osc, ff.rho_gsc, ff.rho_wsc, ff.mu_g, ff.span,
                    d->c_r, d->p_ref_rock, d->gravity};
    fim_status rc = FIM_OK;
#define CK(x)                                                                \
    do {                                                                     \
        rc = (x);                                                            \
        if (rc != FIM_OK) {                                                  \
            g_create_err = m->err;                                           \
            free_all(m);                                                     \
            delete m;                                                        \
            return rc;                                                       \
        }                                                                    \
    } while (0)
    if (hip_stream) {
        m->s = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&m->s) != hipSuccess) {
            g_create_err = "hipStreamCreate failed";
            delete m;
            return FIM_E_HIP;
        }
        m->own_stream = true;
    }
    if (hipEventCreateWithFlags(&m->sync_ev, hipEventDisableTiming) != hipSuccess) {
        g_create_err = "hipEventCreate failed";
        if (m->own_stream) (void)hipStreamDestroy(m->s);
        delete m;
        return FIM_E_HIP;
    }
    // host-side adjacency (both directions, neighbours ascending)
    std::vector<int> deg(n + 1, 0);
    for (int c = 0; c < d->n_conn; c++) {
        deg[d->conn_i[c] + 1]++;
        deg[d->conn_j[c] + 1]++;
    }
    for (int i = 0; i < n; i++) deg[i + 1] += deg[i];
    std::vector<int> nbr(2 * (size_t)d->n_conn);
    std::vector<double> tt(2 * (size_t)d->n_conn);
    {
        std::vector<int> fillp(deg.begin(), deg.end() - 1);
        for (int c = 0; c < d->n_conn; c++) {
            const int a = d->conn_i[c], b = d->conn_j[c];
            nbr[fillp[a]] = b; tt[fillp[a]++] = d->conn_T[c];
            nbr[fillp[b]] = a; tt[fillp[b]++] = d->conn_T[c];
        }
        std::vector<std::pair<int, double>> row;
        for (int i = 0; i < n; i++) {
            row.clear();
            for (int q = deg[i]; q < deg[i + 1]; q++) row.emplace_back(nbr[q], tt[q]);
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int, double>& x, const std::pair<int, double>& y) {
                          return x.first < y.first;
                      });
            for (size_t q = 0; q < row.size(); q++) {
                if (q && row[q].first == row[q - 1].first) {
                    g_create_err = "duplicate connection";
                    free_all(m);
                    delete m;
                    return FIM_E_ARG;
                }
                nbr[deg[i] + q] = row[q].first;
                tt[deg[i] + q] = row[q].second;
            }
            m->max_deg = std::max(m->max_deg, deg[i + 1] - deg[i]);
        }
    }
    std::vector<uint8_t> fl(n, 0);
    std::vector<double> wi(n, 0.0), bh(n, 0.0);
    for (int i = 0; i < n; i++)
        if (d->always_active && d->always_active[i]) fl[i] |= CF_AA;
    for (int p = 0; p < d->n_perf; p++) {
        fl[d->perf_cell[p]] |= CF_PERF;
        wi[d->perf_cell[p]] = d->perf_wi[p];
        bh[d->perf_cell[p]] = d->perf_bhp[p];
    }
    const size_t nn = (size_t)n;
    const size_t nsl = (nn + SLICE - 1) / SLICE;
    m->slot_cap = (long)(m->max_deg + 1) * SLICE * (long)nsl;
    const int B = m->B;
    // the Krylov kernels address the matrix blocks with 32-bit byte offsets
    if ((double)m->slot_cap * B * B * sizeof(double) >= 4294967296.0) {
        g_create_err = "model too large: the matrix blocks would exceed 4 GiB";
        free_all(m);
        delete m;
        return FIM_E_ARG;
    }
    const size_t ntile = std::max((nn + TILE - 1) / TILE, (nsl + TILE - 1) / TILE) + 1;
    CK(dal(m, &m->adj_ptr, nn + 1));
    CK(dal(m, &m->adj_nbr, nbr.size()));
    CK(dal(m, &m->adj_T, tt.size()));
    CK(dal(m, &m->pv, nn));
    CK(dal(m, &m->depth, nn));
    CK(dal(m, &m->wi, nn));
    CK(dal(m, &m->bhp, nn));
    CK(dal(m, &m->flags, nn));
    CK(dal(m, &m->u, nn * B));
    CK(dal(m, &m->un, nn * B));
    CK(dal(m, &m->Mn, nn * B));
    CK(dal(m, &m->dp_abs, nn));
    CK(dal(m, &m->last_dp, nn));
    CK(dal(m, &m->st, nn));
    CK(dal(m, &m->stn, nn));
    CK(dal(m, &m->act, nn));
    CK(dal(m, &m->act2, nn));
    CK(dal(m, &m->lvl, nn));
    CK(dal(m, &m->supp, nn));
    CK(dal(m, &m->bnd, nn));
    CK(dal(m, &m->vt, nn));
    CK(dal(m, &m->outer, nn));
    CK(dal(m, &m->l2g, 2 * nn));
    CK(dal(m, &m->g2l, 2 * nn));
    CK(dal(m, &m->swidth, nsl + 1));
    CK(dal(m, &m->blk, ntile));
    CK(dal(m, &m->col, (size_t)m->slot_cap));
    CK(dal(m, &m->J, (size_t)m->slot_cap * B * B));
    CK(dal(m, &m->F, nn * B));
    CK(dal(m, &m->dinv, nn * B * B));
    // sized for FP64 so that a mixed-precision solve can fall back in place
    CK(dalloc(m, &m->At, (size_t)m->slot_cap * B * B * sizeof(double)));
    CK(dal(m, &m->x64, nn * B));
    CK(dal(m, &m->rir, nn * B));
    CK(dal(m, &m->part, 4 * ((nn * B + NT - 1) / NT + 1)));
    CK(dalloc(m, &m->kvec, 9 * nn * B * sizeof(double)));
    CK(dal(m, &m->xprev, nn * B));
    if (m->o.auto_cut) {
        CK(dal(m, &m->usave, nn * B));
        CK(dal(m, &m->stsave, nn));
        CK(dal(m, &m->suppsave, nn));
    }
    if (d->frac_id) {
        // fracture components (connected over fracture-fracture
        // connections), needed when some fracture cell is not always active
        std::vector<int> comp(n, -1), fc, fcc;
        bool any_loc = false;
        for (int i = 0; i < n; i++) any_loc = any_loc || (d->frac_id[i] >= 0 && !(fl[i] & CF_AA));
        if (any_loc) {
            int nc = 0;
            std::vector<int> todo;
            for (int i = 0; i < n; i++) {
                if (d->frac_id[i] < 0 || comp[i] >= 0) continue;
                comp[i] = nc;
                todo.assign(1, i);
                while (!todo.empty()) {
                    const int a = todo.back();
                    todo.pop_back();
                    for (int q = deg[a]; q < deg[a + 1]; q++) {
                        const int j = nbr[q];
                        if (d->frac_id[j] >= 0 && comp[j] < 0) {
                            comp[j] = nc;
                            todo.push_back(j);
                        }
                    }
                }
                nc++;
            }
            for (int i = 0; i < n; i++)
                if (comp[i] >= 0) {
                    fc.push_back(i);
                    fcc.push_back(comp[i]);
                }
            m->fclose = true;
            m->nfcell = (int)fc.size();
            m->ncomp = nc;
            CK(dal(m, &m->fcells, fc.size()));
            CK(dal(m, &m->fcomp, fc.size()));
            CK(dal(m, &m->ftouch, (size_t)nc));
            HIPX(hipMemcpyAsync(m->fcells, fc.data(), fc.size() * sizeof(int),
                                hipMemcpyHostToDevice, m->s));
            HIPX(hipMemcpyAsync(m->fcomp, fcc.data(), fcc.size() * sizeof(int),
                                hipMemcpyHostToDevice, m->s));
            HIPX(hipStreamSynchronize(m->s));
        }
    }
    std::vector<int> ford;   // fracture-cell ordinal per cell, -1 elsewhere
    std::vector<int> funit;  // fracture cells: unit << 8 | units per block
    if (d->frac_id && m->o.precond != FIM_PC_JACOBI) {
        // (one unknown per cell: the decoupled and coupled blocks coincide)
        m->pc_dec = m->o.precond == FIM_PC_FRACTURE && m->fk > 1;
        ford.assign(n, -1);
        int nfc = 0;
        for (int i = 0; i < n; i++)
            if (d->frac_id[i] >= 0) ford[i] = nfc++;
        if (nfc > 0) {
            m->pc_cap = pc_cells(B);
            if (!fracture_units(n, d->frac_id, deg, nbr, m->pc_cap, funit)) {
                g_create_err = "model too large: a fracture has more than 2^23 cells";
                free_all(m);
                delete m;
                return FIM_E_ARG;
            }
            const double store = (double)nfc * pc_cell_stride(B) * sizeof(float);
            if (store >= 4294967296.0) {
                g_create_err = "model too large: fracture-block inverses would exceed 4 GiB";
                free_all(m);
                delete m;
                return FIM_E_ARG;
            }
            CK(dal(m, &m->frac_id, nn));
            CK(dal(m, &m->ford, nn));
            CK(dal(m, &m->funit, nn));
            CK(dal(m, &m->pcinfo, nn));
            CK(dal(m, &m->pcoff, nn));
            CK(dal(m, &m->pcM, (size_t)nfc * pc_cell_stride(B)));
            // blocks have >= 2 rows, all fracture cells
            CK(dal(m, &m->pclist, 2 * (nfc / 2 + 1)));
            // about as many single-wave workgroups as fit at once (LDS)
            // resident single-wave workgroups per CU (LDS-bound: 8 with
            // coupled blocks, about 20 with the decoupled blocks' rows)
            m->pc_inv_grid = std::min(nfc / 2 + 1, (m->pc_dec ? 20 : 8) * m->cus);
            m->pc_nfc = nfc;
            m->use_pc = true;
        }
    }
    CK(dal(m, &m->sc, 1));
    CK(dal(m, &m->part_ir, 14 * KB_MAXB));
    CK(dal(m, &m->ns, 1));
    CK(dal(m, &m->dint, 8));
    CK(dal(m, &m->dsub, 1024));
    if (hipHostMalloc((void**)&m->hsc, sizeof(KScal)) != hipSuccess ||
        hipHostMalloc((void**)&m->hns, sizeof(NStat), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostMalloc((void**)&m->hint, 8 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&m->hns_dev, m->hns, 0) != hipSuccess ||
        hipHostGetDevicePointer((void**)&m->hint_dev, m->hint, 0) != hipSuccess ||
        hipHostMalloc((void**)&m->hsub, 1024 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&m->hpart, 2 * KB_MAXB * sizeof(double)) != hipSuccess) {
        m->err = "hipHostMalloc failed";
        CK(FIM_E_NOMEM);
    }
    // the allocation-free iteration: this device's scratch address (looked
    // up once per device) and the pinned parts of its solve table
    CK(table_alloc_host(m, m->nat, 1));
    {
        std::string why;
        m->scratch = n <= NA_MAX_CELLS ? scratch_address(m->dev, &why) : nullptr;
        if (m->scratch) {
            m->nat.dsegs = (KSeg*)(m->scratch + NA_OFF_SEGS);
            m->nat.dblk = (int*)(m->scratch + NA_OFF_BMAP);
        }
    }
    auto up = [&](void* dst, const void* src, size_t bytes) -> fim_status {
        if (!bytes) return FIM_OK;
        HIPX(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, m->s));
        return FIM_OK;
    };
    CK(up(m->adj_ptr, deg.data(), (nn + 1) * sizeof(int)));
    CK(up(m->adj_nbr, nbr.data(), nbr.size() * sizeof(int)));
    CK(up(m->adj_T, tt.data(), tt.size() * sizeof(double)));
    CK(up(m->pv, d->pv_ref, nn * sizeof(double)));
    CK(up(m->depth, d->depth, nn * sizeof(double)));
    CK(up(m->wi, wi.data(), nn * sizeof(double)));
    CK(up(m->bhp, bh.data(), nn * sizeof(double)));
    CK(up(m->flags, fl.data(), nn));
    if (m->use_pc) {
        CK(up(m->frac_id, d->frac_id, nn * sizeof(int)));
        CK(up(m->ford, ford.data(), nn * sizeof(int)));
        CK(up(m->funit, funit.data(), nn * sizeof(int)));
    }
    // zero the counters and state
    std::vector<char> z(std::max(sizeof(KScal), sizeof(NStat)), 0);
    CK(up(m->sc, z.data(), sizeof(KScal)));
    CK(up(m->ns, z.data(), sizeof(NStat)));
    launch_fill_f64(m->u, (long)nn * B, 0.0, m->s);
    launch_fill_u8((uint8_t*)m->st, n, 0, m->s);
    launch_fill_i32(m->dint, 8, 0, m->s);
    if (hipStreamSynchronize(m->s) != hipSuccess) {
        m->err = "initial upload failed";
        CK(FIM_E_HIP);
    }
    m->g = Graph{n, m->adj_ptr, m->adj_nbr, m->adj_T, m->pv, m->depth, m->flags, m->wi, m->bhp};
#undef CK
    *out = m;
    return FIM_OK;
}

fim_status fim_destroy_model(fim_model* m) {
    if (!m) return FIM_E_ARG;
    if (m->s) (void)hipStreamSynchronize(m->s);
    for (fim_model* c : m->dd_clones) free_clone(c);
    m->dd_clones.clear();
    table_free(m->dd_tab);
    free_all(m);
    delete m;
    return FIM_OK;
}

fim_status fim_set_state(fim_model* m, const double* u, const int8_t* status, int mem) {
    if (!m || !u) return FIM_E_ARG;
    const size_t nb = (size_t)m->n * m->B;
    std::vector<double> hu;
    const double* src = u;
    if (mem == FIM_DEVICE) {
        hu.resize(nb);
        HIPX(hipMemcpyAsync(hu.data(), u, nb * sizeof(double), hipMemcpyDeviceToHost, m->s));
        HIPX(hipStreamSynchronize(m->s));
        src = hu.data();
    }
    for (size_t q = 0; q < nb; q++)
        if (!std::isfinite(src[q])) {
            m->err = "non-finite state value";
            return FIM_E_NONFINITE;
        }
    const hipMemcpyKind kind = mem == FIM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPX(hipMemcpyAsync(m->u, u, nb * sizeof(double), kind, m->s));
    if (status) HIPX(hipMemcpyAsync(m->st, status, m->n, kind, m->s));
    else launch_fill_u8((uint8_t*)m->st, m->n, 0, m->s);
    HIPX(hipStreamSynchronize(m->s));
    m->in_step = false;
    m->have_history = false;
    m->inspect_ready = false;
    return FIM_OK;
}

fim_status fim_get_state(fim_model* m, double* u_out, int8_t* status_out, int mem) {
    if (!m || !u_out) return FIM_E_ARG;
    const hipMemcpyKind kind = mem == FIM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPX(hipMemcpyAsync(u_out, m->u, (size_t)m->n * m->B * sizeof(double), kind, m->s));
    if (status_out) HIPX(hipMemcpyAsync(status_out, m->st, m->n, kind, m->s));
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

// ------------------------------------------------------------ checkpoints
// Blob: header, the state (b planes of n doubles), the phase status (n
// bytes) and the previous step's support set (n bytes, zero without one).
struct CkptHead {
    char magic[8];
    int32_t version, n, b, have_history;
};
static const char CKPT_MAGIC[8] = {'F', 'I', 'M', 'C', 'K', 'P', 'T', '1'};

int64_t fim_checkpoint_bytes(const fim_model* m) {
    if (!m) return -1;
    return (int64_t)sizeof(CkptHead) + (int64_t)m->n * m->B * 8 + 2 * (int64_t)m->n;
}

fim_status fim_get_checkpoint(fim_model* m, void* buf, int64_t cap) {
    if (!m || !buf) return FIM_E_ARG;
    if (cap < fim_checkpoint_bytes(m)) {
        m->err = "checkpoint buffer smaller than fim_checkpoint_bytes";
        return FIM_E_ARG;
    }
    if (m->in_step) {
        m->err = "checkpoints are taken between timesteps";
        return FIM_E_STATE;
    }
    CkptHead h{};
    std::memcpy(h.magic, CKPT_MAGIC, 8);
    h.version = 1;
    h.n = m->n;
    h.b = m->B;
    h.have_history = m->have_history ? 1 : 0;
    char* p = (char*)buf;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t nu = (size_t)m->n * m->B * sizeof(double);
    HIPX(hipMemcpyAsync(p, m->u, nu, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(p + nu, m->st, m->n, hipMemcpyDeviceToHost, m->s));
    if (m->have_history)
        HIPX(hipMemcpyAsync(p + nu + m->n, m->supp, m->n, hipMemcpyDeviceToHost, m->s));
    else
        std::memset(p + nu + m->n, 0, m->n);
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

fim_status fim_set_checkpoint(fim_model* m, const void* buf, int64_t len) {
    if (!m || !buf) return FIM_E_ARG;
    CkptHead h{};
    if (len < (int64_t)sizeof h) {
        m->err = "checkpoint too short";
        return FIM_E_ARG;
    }
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != 1) {
        m->err = "not a checkpoint of this library";
        return FIM_E_ARG;
    }
    if (h.n != m->n || h.b != m->B || len < fim_checkpoint_bytes(m)) {
        m->err = "checkpoint of another model shape";
        return FIM_E_ARG;
    }
    const char* p = (const char*)buf + sizeof h;
    const size_t nu = (size_t)m->n * m->B * sizeof(double);
    TRY(fim_set_state(m, (const double*)p, (const int8_t*)(p + nu), FIM_HOST));
    if (h.have_history) {
        HIPX(hipMemcpyAsync(m->supp, p + nu + m->n, m->n, hipMemcpyHostToDevice, m->s));
        HIPX(hipStreamSynchronize(m->s));
        m->have_history = true;
    }
    return FIM_OK;
}

// After the update of an Algorithm 1 / full iteration: the set update and
// compaction for the next iteration and the status copies (launch only).
static fim_status newton_post_launch(fim_model* m) {
    if (m->step_mode == FIM_LOCAL) {
        const int pi = pbeg(m, PK_SETS);
        launch_fill_i32(m->dint, 1, 0, m->s);
        launch_mark_expand(m->nA, m->l2g, m->bnd, m->dp_abs, m->o.eps_loc, m->o.m_layers, m->g,
                           m->act, nullptr, m->dint, m->lvl, m->s);
        launch_shrink(m->nA, m->l2g, m->dp_abs, m->o.eps_loc, m->g, m->act, m->dint, m->s);
        frac_closure(m);
        compact(m);
        pend(m, pi, m->n);
    } else if (m->step_mode == FIM_RESID) {
        // error measure at the updated state on every cell (into last_dp,
        // unused outside Algorithm 2), the unconverged cells and their
        // neighbour layers; dint[0] = number of unconverged cells
        const int pi = pbeg(m, PK_SETS);
        launch_resid_err(m->fk, m->n, m->g, m->f, m->u, m->st, m->Mn, m->step_dt, m->last_dp,
                         m->s);
        launch_fill_i32(m->dint, 1, 0, m->s);
        launch_mark_resid(m->n, m->last_dp, m->o.eps_res, m->o.res_layers, m->g, m->act,
                          m->dint, m->lvl, m->s);
        compact(m);
        pend(m, pi, m->n);
        m->full_ready = false;   // l2g / g2l now hold the new set
    }
    launch_status_out(m->ns, m->dint, m->hns_dev, m->hint_dev, m->s);
    return FIM_OK;
}

// The decisions of the iteration, once the status copies have landed.
// defer (batched iterations): instead of launching the next iteration's
// structure pass or the converged step's support, report that they are
// due (the new n_A is set).
struct BatchDefer {
    bool structure = false, commit = false;
};
static fim_status newton_post_finish(fim_model* m, fim_iter_stats* it,
                                     BatchDefer* defer = nullptr) {
    if (defer) *defer = BatchDefer();
    const bool local = m->step_mode == FIM_LOCAL;
    const NStat ns = *m->hns;
    m->nu++;
    const bool conv = converged(m, ns);
    if (it) {
        // dint[2] still holds |V_B| of this iteration (the next boundary
        // pass runs after this readback)
        it->n_boundary = local ? m->hint[2] : 0;
        it->dp_max = ns.dp_max;
        it->ds_max = ns.ds_max;
        it->n_switch = ns.nswitch;
        it->nonfinite = ns.nonfinite;
    }
    if (ns.nonfinite) {
        TRY(rollback(m));
        m->err = "non-finite update";
        return FIM_NOT_CONVERGED;
    }
    const bool resid = m->step_mode == FIM_RESID;
    bool done;
    if (local) {
        m->is_expand = m->hint[0] != 0;
        done = conv && !m->is_expand;
        if (it) it->is_expand = m->is_expand;
    } else if (resid) {
        done = conv || m->hint[0] == 0;   // or no cell left unconverged
    } else {
        done = conv;
    }
    if (done) {
        if (defer) {
            m->have_history = true;
            m->in_step = false;
            defer->commit = true;
        } else {
            commit(m);
        }
        if (it) it->converged = 1;
        return FIM_OK;
    }
    if (m->nu >= m->o.max_newton) {
        TRY(rollback(m));
        m->err = "Newton iteration cap reached";
        return FIM_NOT_CONVERGED;
    }
    if ((local || resid) && defer) {
        m->nA = m->hint[1];
        defer->structure = true;
    } else if (local) {
        m->nA = m->hint[1];
        const int pi = pbeg(m, PK_SETS);
        TRY(structure(m));
        launch_fill_i32(&m->dint[2], 1, 0, m->s);
        launch_boundary(m->nA, m->l2g, m->g2l, m->g, m->bnd, &m->dint[2], m->s);
        pend(m, pi, m->nA);
    } else if (resid) {
        m->nA = m->hint[1];
        const int pi = pbeg(m, PK_SETS);
        TRY(structure(m));
        pend(m, pi, m->nA);
    }
    return FIM_OK;
}

// An iteration on an empty active set (Algorithm 1 or 2 on a model with
// no always-active cells and an empty previous support) has nothing to
// solve: du = 0, which meets the convergence test, so the step ends with
// u^n unchanged after this one iteration.
static fim_status empty_iteration(fim_model* m, fim_iter_stats* it) {
    m->nu++;
    if (m->flags_on) launch_fill_u8(m->classes, m->n, 0, m->s);
    commit(m);
    if (it) {
        it->n_active = 0;
        it->converged = 1;
    }
    return FIM_OK;
}

static fim_status newton_full_or_local(fim_model* m, fim_iter_stats* it) {
    if (m->nA == 0) return empty_iteration(m, it);
    TRY(local_newton(m, it));
    TRY(newton_post_launch(m));
    HIPX(spin_sync(m, m->s));
    pflush(m);
    return newton_post_finish(m, it);
}

// One sweep of the additive phase 2 (FIM_DD_ADD): the pending subdomains
// (subdomain maxima already in hsub) are activated in workspaces, assembled
// from the same state, solved together in one batched linear solve, and
// each cell takes the update of the first subdomain that contains it.
static fim_status dd_additive_sweep(fim_model* m, int N, fim_iter_stats* it) {
    std::vector<int> todo;
    for (int k = 0; k < N; k++)
        if (m->hsub[k] >= m->o.eps_loc) todo.push_back(k);
    if (todo.empty()) {
        commit(m);
        if (it) it->converged = 1;
        return FIM_OK;
    }
    const int P = (int)todo.size();
    m->dd_sweeps++;
    if (m->dd_sweeps > m->o.max_sweeps || m->nu + P > m->o.max_newton * 8) {
        TRY(rollback(m));
        m->err = "Algorithm 2 sweep cap reached";
        return FIM_NOT_CONVERGED;
    }
    while ((int)m->dd_clones.size() < P) {
        fim_model* c = nullptr;
        TRY(make_clone(m, &c));
        m->dd_clones.push_back(c);
    }
    if (m->dd_tab.cap < P) {
        table_free(m->dd_tab);
        TRY(table_alloc(m, m->dd_tab, std::max(P, 4)));
    }
    std::vector<fim_model*> ws(m->dd_clones.begin(), m->dd_clones.begin() + P);
    long sum_n = 0;
    for (int j = 0; j < P; j++) {
        fim_model* c = ws[j];
        const DDSub& sd = m->subs[todo[j]];
        c->s = m->s;
        c->step_dt = m->step_dt;
        c->step_mode = m->step_mode;
        c->ew_owner = m;        // the subdomain's forcing sequence
        c->dd_cur = todo[j];
        launch_fill_u8(c->act, c->n, 0, c->s);
        launch_scatter_flags(sd.cells_n, m->sd_cells + sd.cells_off, c->act, c->s);
        compact(c);
        c->nA = sd.cells_n;
        TRY(structure(c));
        newton_assemble(c);
        solve_prep(c, c->s);
        sum_n += sd.cells_n;
    }
    const fim_status sv = solve_batch(ws, m->dd_tab, m->s, true);
    for (fim_model* c : ws) c->dd_cur = -1;
    TRY(sv);
    int kry = 0;
    for (int j = 0; j < P; j++) {
        fim_model* c = ws[j];
        launch_update(c->fk, c->nA, c->l2g, c->x64, c->u, c->st, c->n, c->f, c->o.ds_max,
                      c->dp_abs, c->part, c->ns, c->s, m->dd_owner, todo[j]);
        launch_copy_owned(c->nA, c->l2g, m->dd_owner, todo[j], c->dp_abs, m->last_dp, c->s);
        HIPX(hipMemcpyAsync(c->hns, c->ns, sizeof(NStat), hipMemcpyDeviceToHost, c->s));
        kry += c->last_kry;
    }
    HIPX(spin_sync(m, m->s));
    m->nu += P;
    double dpm = 0.0, dsm = 0.0;
    bool bad = false;
    for (int j = 0; j < P; j++) {
        const NStat& ns = *ws[j]->hns;
        dpm = std::max(dpm, ns.dp_max);
        dsm = std::max(dsm, ns.ds_max);
        bad = bad || ns.nonfinite;
    }
    m->sum_active += (double)sum_n;
    m->max_active = std::max(m->max_active, (int)std::min<long>(sum_n, INT_MAX));
    m->step_kry += kry;
    if (it) {
        it->n_active = (int)std::min<long>(sum_n, INT_MAX);
        it->subdomain = P;
        it->krylov_iters = kry;
        it->dp_max = dpm;
        it->ds_max = dsm;
        it->nonfinite = bad ? 1 : 0;
    }
    if (bad) {
        TRY(rollback(m));
        m->err = "non-finite update";
        return FIM_NOT_CONVERGED;
    }
    return FIM_OK;
}

// one inner iteration of Algorithm 2
static fim_status newton_dd(fim_model* m, fim_iter_stats* it) {
    if (it) it->phase = m->dd_phase;
    if (m->dd_phase == 1 && m->nA == 0) return empty_iteration(m, it);
    if (m->dd_phase == 1) {
        // at most max_newton subdomain-building solves
        if (m->nu >= m->o.max_newton) {
            TRY(rollback(m));
            m->err = "Algorithm 2 built subdomains for max_newton iterations";
            return FIM_NOT_CONVERGED;
        }
        if (it) it->subdomain = (int)m->subs.size();
        TRY(local_newton(m, it));
        launch_copy_masked(m->nA, m->l2g, m->dp_abs, m->last_dp, m->s);
        TRY(dd_store(m));
        if (m->step_mode == FIM_DD_ADD) {
            const DDSub& sd = m->subs.back();
            launch_set_owner(sd.cells_n, m->sd_cells + sd.cells_off, m->dd_owner,
                             (int)m->subs.size() - 1, m->s);
        }
        HIPX(hipMemcpyAsync(m->hns, m->ns, sizeof(NStat), hipMemcpyDeviceToHost, m->s));
        bool expand = false;
        TRY(dd_expand_sets(m, m->o.eps_loc, m->o.m_layers_dd, &expand));
        m->nu++;
        const NStat ns = *m->hns;
        if (it) { it->dp_max = ns.dp_max; it->ds_max = ns.ds_max; it->nonfinite = ns.nonfinite; }
        if (ns.nonfinite) {
            TRY(rollback(m));
            m->err = "non-finite update";
            return FIM_NOT_CONVERGED;
        }
        if (expand) {
            if (it) it->is_expand = 1;
        } else {
            m->dd_phase = 2;
            m->dd_next = 0;
            // the multiplicative search counts its first sweep here, each
            // additive call counts its own
            m->dd_sweeps = m->step_mode == FIM_DD_ADD ? 0 : 1;
        }
    } else {
        const int N = (int)m->subs.size();
        // find the next subdomain (in sweep order) whose update or whose
        // outer-layer boundary values are not negligible
        launch_sub_max(N, m->subs.data(), m->sd_cells, m->sd_outer, m->last_dp, m->dsub, m->s);
        TRY(sync_read(m, m->hsub, m->dsub, N * sizeof(double)));
        if (m->step_mode == FIM_DD_ADD) return dd_additive_sweep(m, N, it);
        bool new_sweep = false;
        const int pick = dd_pick(m->hsub, N, m->o.eps_loc, m->dd_next, &new_sweep);
        if (pick < 0) {
            commit(m);
            if (it) it->converged = 1;
            return FIM_OK;
        }
        if (new_sweep) m->dd_sweeps++;
        if (m->dd_sweeps > m->o.max_sweeps || m->nu >= m->o.max_newton * 8) {
            TRY(rollback(m));
            m->err = "Algorithm 2 sweep cap reached";
            return FIM_NOT_CONVERGED;
        }
        if (it) it->subdomain = pick;
        TRY(dd_activate(m, pick));
        m->dd_cur = pick;
        const fim_status ln = local_newton(m, it);
        m->dd_cur = -1;
        TRY(ln);
        launch_copy_masked(m->nA, m->l2g, m->dp_abs, m->last_dp, m->s);
        HIPX(hipMemcpyAsync(m->hns, m->ns, sizeof(NStat), hipMemcpyDeviceToHost, m->s));
        HIPX(spin_sync(m, m->s));
        m->nu++;
        const NStat ns = *m->hns;
        if (it) { it->dp_max = ns.dp_max; it->ds_max = ns.ds_max; it->nonfinite = ns.nonfinite; }
        if (ns.nonfinite) {
            TRY(rollback(m));
            m->err = "non-finite update";
            return FIM_NOT_CONVERGED;
        }
        m->dd_next = pick + 1;    // N after the last subdomain: the next pick wraps
        m->dd_k = pick;
    }
    return FIM_OK;
}

fim_status fim_newton_step(fim_model* m, double dt, int mode, fim_iter_stats* it) {
    if (!m) return FIM_E_ARG;
    if (!(dt > 0.0) || !std::isfinite(dt) || mode < FIM_FULL || mode > FIM_DD_ADD) {
        m->err = "dt must be positive and mode FULL, LOCAL, DD, RESID or DD_ADD";
        return FIM_E_ARG;
    }
    if (it) std::memset(it, 0, sizeof(*it));
    if (m->in_step && (dt != m->step_dt || mode != m->step_mode)) {
        m->err = "dt or mode changed inside a timestep";
        return FIM_E_STATE;
    }
    if (!m->in_step) TRY(begin_step(m, dt, mode));
    return (mode == FIM_DD || mode == FIM_DD_ADD) ? newton_dd(m, it)
                                                   : newton_full_or_local(m, it);
}

// For the duration of one allocation-free call: the kernels' partial
// sums, Krylov scalars, compaction tile counts and the solve table come
// from this device's scratch array instead of the model's own buffers.
struct NoallocScope {
    fim_model* m;
    double* part_ir;
    KScal* sc;
    int* blk;
    double* part;
    explicit NoallocScope(fim_model* mm)
        : m(mm), part_ir(mm->part_ir), sc(mm->sc), blk(mm->blk), part(mm->part) {
        m->part_ir = (double*)(m->scratch + NA_OFF_PART);
        m->sc = (KScal*)(m->scratch + NA_OFF_SC);
        m->blk = (int*)(m->scratch + NA_OFF_TILES);
        m->part = (double*)(m->scratch + NA_OFF_UPART);
        m->noalloc = true;
    }
    ~NoallocScope() {
        m->part_ir = part_ir;
        m->sc = sc;
        m->blk = blk;
        m->part = part;
        m->noalloc = false;
    }
    NoallocScope(const NoallocScope&) = delete;
    NoallocScope& operator=(const NoallocScope&) = delete;
};

fim_status fim_newton_step_noalloc(fim_model* m, double dt, int mode, fim_iter_stats* it) {
    if (!m) return FIM_E_ARG;
    if (m->n > NA_MAX_CELLS) {
        m->err = "fim_newton_step_noalloc: the model has " + std::to_string(m->n) +
                 " cells, more than the " + std::to_string(NA_MAX_CELLS) +
                 " its scratch array is sized for";
        return FIM_E_ARG;
    }
    if (mode == FIM_DD || mode == FIM_DD_ADD) {
        m->err = "fim_newton_step_noalloc runs FIM_FULL, FIM_LOCAL or FIM_RESID "
                 "(Algorithm 2 grows its subdomain lists)";
        return FIM_E_ARG;
    }
    if (m->prof.on) {
        m->err = "fim_newton_step_noalloc: the event profiler creates events; disable it";
        return FIM_E_STATE;
    }
    if (!m->scratch) {
        std::string why;
        (void)scratch_address(m->dev, &why);
        m->err = "fim_newton_step_noalloc: no scratch address on this device: " + why;
        return FIM_E_HIP;
    }
    NoallocScope scope(m);
    // the scratch array keeps the previous call's contents: the Krylov
    // scalars start from zero (every other part is written before it is read)
    launch_fill_i32((int*)m->sc, (int)(sizeof(KScal) / sizeof(int)), 0, m->s);
    return fim_newton_step(m, dt, mode, it);
}

static fim_status solve_once(fim_model* m, double dt, int mode, fim_step_stats* st) {
    fim_iter_stats it;
    for (;;) {
        fim_status r = fim_newton_step(m, dt, mode, &it);
        // Algorithm 2's last call finds no subdomain to solve: no iteration
        const bool solved =
            !((mode == FIM_DD || mode == FIM_DD_ADD) && it.phase == 2 && it.n_active == 0);
        if (st) {
            st->iterations += solved ? 1 : 0;
            st->krylov_iters += it.krylov_iters;
            st->sum_active += it.n_active;
            st->max_active = std::max(st->max_active, it.n_active);
        }
        if (r != FIM_OK) return r;
        if (it.converged) {
            if (st) {
                st->converged = 1;
                st->subdomains = (int)m->subs.size();
            }
            return FIM_OK;
        }
    }
}

fim_status fim_solve_timestep(fim_model* m, double dt, int mode, fim_step_stats* st) {
    if (!m) return FIM_E_ARG;
    if (st) std::memset(st, 0, sizeof(*st));
    if (m->in_step) {
        m->err = "a timestep is already in progress";
        return FIM_E_STATE;
    }
    const size_t nb = (size_t)m->n * m->B;
    const bool had_history = m->have_history;
    if (m->o.auto_cut) {
        // substeps that succeed are committed one by one; a later failure
        // must still leave the model at u^n of this call
        HIPX(hipMemcpyAsync(m->usave, m->u, nb * sizeof(double), hipMemcpyDeviceToDevice, m->s));
        HIPX(hipMemcpyAsync(m->stsave, m->st, m->n, hipMemcpyDeviceToDevice, m->s));
        HIPX(hipMemcpyAsync(m->suppsave, m->supp, m->n, hipMemcpyDeviceToDevice, m->s));
    }
    fim_status r = solve_once(m, dt, mode, st);
    if (r != FIM_NOT_CONVERGED || !m->o.auto_cut) return r;
    // halve dt and substep; each substep may be cut further
    std::vector<std::pair<double, int>> todo{{dt * 0.5, 1}, {dt * 0.5, 1}};
    while (!todo.empty()) {
        auto [h, depth] = todo.front();
        todo.erase(todo.begin());
        if (st) st->cuts = std::max(st->cuts, depth);
        r = solve_once(m, h, mode, st);
        if (r == FIM_OK) continue;
        if (r == FIM_NOT_CONVERGED && depth < m->o.max_cuts) {
            todo.insert(todo.begin(), {{h * 0.5, depth + 1}, {h * 0.5, depth + 1}});
            continue;
        }
        if (r == FIM_NOT_CONVERGED) {
            const std::string why = m->err;
            HIPX(hipMemcpyAsync(m->u, m->usave, nb * sizeof(double), hipMemcpyDeviceToDevice, m->s));
            HIPX(hipMemcpyAsync(m->st, m->stsave, m->n, hipMemcpyDeviceToDevice, m->s));
            HIPX(hipMemcpyAsync(m->supp, m->suppsave, m->n, hipMemcpyDeviceToDevice, m->s));
            HIPX(hipStreamSynchronize(m->s));
            m->have_history = had_history;
            m->in_step = false;
            if (st) st->converged = 0;
            m->err = "timestep cut limit reached (" + why + "); state restored to u^n";
        }
        return r;
    }
    if (st) st->converged = 1;
    return FIM_OK;
}

// ---------------------------------------------------------- footprint
int64_t fim_model_bytes(const fim_model* m) { return m ? (int64_t)m->bytes : 0; }

int64_t fim_estimate_bytes(const fim_model_desc* d, const fim_options* o) {
    if (!d || d->n_cells <= 0) return -1;
    const size_t n = (size_t)d->n_cells;
    const size_t B = (size_t)d->fluid.kind;
    std::vector<int> deg(n, 0);
    for (int c = 0; c < d->n_conn; c++) {
        if (d->conn_i[c] < 0 || d->conn_j[c] >= d->n_cells) return -1;
        deg[d->conn_i[c]]++;
        deg[d->conn_j[c]]++;
    }
    int maxdeg = 0;
    for (size_t i = 0; i < n; i++) maxdeg = std::max(maxdeg, deg[i]);
    const size_t nsl = (n + SLICE - 1) / SLICE;
    const size_t slots = (size_t)(maxdeg + 1) * SLICE * nsl;
    const size_t nc2 = 2 * (size_t)d->n_conn;
    size_t b = 0;
    b += (n + 1) * 4 + nc2 * 12;                  // adjacency
    b += n * (8 * 4 + 1);                         // pv, depth, wi, bhp, flags
    b += n * B * 8 * 3 + n * 8 * 2 + n * 2;       // u, un, Mn, dp_abs, last_dp, status
    b += n * 7;                                   // byte flags, marking levels
    b += n * 4 * 4 + nsl * 4;                     // l2g, g2l (2n each), swidth
    b += slots * (4 + B * B * 8 + B * B * 8);     // col, J, A~ (sized for FP64)
    b += n * B * (8 + B * 8);                     // F, dinv
    b += n * B * 8 * 3 + n * B * 8 * 9;           // x64, xprev, rir, Krylov vectors
    b += 4 * (n * B / NT + 2) * 8 + 8 * KB_MAXB * 8;
    if (o && o->auto_cut) b += n * B * 8 + 2 * n;   // entry snapshot of auto_cut
    if (d->frac_id) {
        // fracture-component lists of localized fracture cells (at most)
        size_t nfc = 0;
        bool loc = false;
        for (size_t i = 0; i < n; i++)
            if (d->frac_id[i] >= 0) {
                nfc++;
                loc = loc || !(d->always_active && d->always_active[i]);
            }
        if (loc) b += nfc * 9;
    }
    const int pc = o ? o->precond : FIM_PC_FRACTURE;
    if (d->frac_id && pc != FIM_PC_JACOBI) {
        size_t nfc = 0;
        for (size_t i = 0; i < n; i++) nfc += d->frac_id[i] >= 0 ? 1 : 0;
        if (nfc) b += n * 20 + nfc * (size_t)pc_cell_stride(B) * 4 + (nfc / 2 + 1) * 8;
    }
    return (int64_t)b;
}

// ------------------------------------------------------------- batches
struct fim_batch {
    std::vector<fim_model*> ms;
    std::vector<hipEvent_t> ev;   // one per member: stream hand-over
    hipEvent_t done_ev = nullptr;
    hipStream_t s = nullptr;
    bool own_stream = false;
    SolveTable tab;
    int B = 0, precision = 0;
    std::string err;
    // member tables of the segmented launches, uploaded alternately into
    // two slots (ev: the upload that last read a slot's host half)
    struct Slot {
        char* h = nullptr;
        char* d = nullptr;
        size_t host_bytes = 0, dev_bytes = 0;
        hipEvent_t ev = nullptr;
    } slot[2];
    int cur = 0;
    BStatus* hstat = nullptr;   // per member status words (pinned, mapped)
    BStatus* dstat = nullptr;
    int stat_cap = 0;
};

// Layout of a slot for K members whose cells need at most W cell
// workgroups in all: host part = the BMember table and the three prefix
// arrays; device part = the same plus the four workgroup maps.
static int bt_blocks(long n) { return (int)((n + NT - 1) / NT); }
static size_t bt_pref_off(int K) { return ((size_t)K * sizeof(BMember) + 255) / 256 * 256; }
static size_t bt_host_bytes(int K) { return bt_pref_off(K) + 3 * (size_t)(K + 1) * sizeof(int); }
static size_t bt_map_off(int K) { return (bt_host_bytes(K) + 255) / 256 * 256; }
static size_t bt_dev_bytes(int K, long W) {
    return bt_map_off(K) + (size_t)(3 * W + K) * sizeof(BMap);
}

static void batch_tables_free(fim_batch* b) {
    for (auto& sl : b->slot) {
        if (sl.ev) (void)hipEventSynchronize(sl.ev);
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.d) (void)hipFree(sl.d);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        sl = fim_batch::Slot();
    }
    if (b->hstat) (void)hipHostFree(b->hstat);
    b->hstat = b->dstat = nullptr;
    b->stat_cap = 0;
}

// sized for the members of the batch (all of them live at most)
static fim_status batch_tables_alloc(fim_batch* b) {
    const int K = (int)b->ms.size();
    long W = 0;
    for (fim_model* m : b->ms) W += bt_blocks(m->n);
    const size_t hb = bt_host_bytes(K), db = bt_dev_bytes(K, W);
    for (auto& sl : b->slot) {
        if (sl.host_bytes >= hb && sl.dev_bytes >= db) continue;
        if (sl.ev) (void)hipEventSynchronize(sl.ev);
        if (sl.h) (void)hipHostFree(sl.h);
        if (sl.d) (void)hipFree(sl.d);
        sl.h = sl.d = nullptr;
        sl.host_bytes = sl.dev_bytes = 0;
        if (hipHostMalloc((void**)&sl.h, hb) != hipSuccess ||
            hipMalloc((void**)&sl.d, db) != hipSuccess) {
            b->err = "batch table allocation failed";
            return FIM_E_NOMEM;
        }
        sl.host_bytes = hb;
        sl.dev_bytes = db;
        if (!sl.ev && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
            b->err = "hipEventCreate failed";
            return FIM_E_HIP;
        }
    }
    if (b->stat_cap < K) {
        if (b->hstat) (void)hipHostFree(b->hstat);
        b->hstat = b->dstat = nullptr;
        b->stat_cap = 0;
        if (hipHostMalloc((void**)&b->hstat, (size_t)K * sizeof(BStatus),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer((void**)&b->dstat, b->hstat, 0) != hipSuccess) {
            b->err = "pinned status buffer not available";
            return FIM_E_NOMEM;
        }
        b->stat_cap = K;
    }
    return FIM_OK;
}

// One member as the segmented kernels see it (its current n_A and step).
static BMember bmember(fim_model* m) {
    BMember x;
    std::memset(&x, 0, sizeof(x));
    x.ls = lsys(m);
    x.g = m->g;
    x.f = m->f;
    x.u = m->u;
    x.st = m->st;
    x.Mn = m->Mn;
    x.un = m->un;
    x.stn = m->stn;
    x.supp = m->supp;
    x.dt = m->step_dt;
    x.inv_dt = 1.0 / m->step_dt;
    x.ds_max = m->o.ds_max;
    x.dinv = m->dinv;
    x.At = m->At;
    x.x64 = m->x64;
    x.dp_abs = m->dp_abs;
    x.part = m->part;
    x.ns = m->ns;
    x.act = m->act;
    x.bnd = m->bnd;
    x.lvl = m->lvl;
    x.dint = m->dint;
    x.blk = m->blk;
    x.last_dp = m->last_dp;
    x.eps_loc = m->o.eps_loc;
    x.eps_res = m->o.eps_res;
    if (m->use_pc) {
        x.frac_id = m->frac_id;
        x.ford = m->ford;
        x.funit = m->funit;
        x.pcinfo = m->pcinfo;
        x.pcoff = m->pcoff;
        x.pclist = m->pclist;
    }
    x.n = m->n;
    x.nA = m->nA;
    x.mode = m->step_mode;
    x.layers = m->step_mode == FIM_LOCAL ? std::min(m->o.m_layers, MAX_LAYERS)
             : m->step_mode == FIM_RESID ? std::min(m->o.res_layers, MAX_LAYERS) : 0;
    x.compact = m->step_mode != FIM_FULL ? 1 : 0;
    return x;
}

// The device table and workgroup maps of one phase of a batched call.
struct BPhase {
    const BMember* t = nullptr;
    const BMap *rows = nullptr, *cells = nullptr, *tiles = nullptr, *mem = nullptr;
    int K = 0, nrows = 0, ncells = 0, ntiles = 0, layers = 0;
    bool any_resid = false;
};

static fim_status batch_upload(fim_batch* b, const std::vector<BMember>& ent, BPhase& ph) {
    const int K = (int)ent.size();
    fim_batch::Slot& sl = b->slot[b->cur];
    b->cur ^= 1;
    if (hipEventSynchronize(sl.ev) != hipSuccess) {
        b->err = "hipEventSynchronize failed";
        return FIM_E_HIP;
    }
    BMember* t = (BMember*)sl.h;
    int* pref = (int*)(sl.h + bt_pref_off(K));
    int acc[3] = {0, 0, 0};
    ph = BPhase();
    ph.K = K;
    for (int q = 0; q < K; q++) {
        t[q] = ent[q];
        const int n = t[q].n;
        const int c[3] = {bt_blocks(std::max(t[q].nA, 0)), bt_blocks(n), (n + TILE - 1) / TILE};
        for (int k = 0; k < 3; k++) {
            pref[k * (K + 1) + q] = acc[k];
            acc[k] += c[k];
        }
        ph.layers = std::max(ph.layers, t[q].layers);
        ph.any_resid = ph.any_resid || t[q].mode == FIM_RESID;
    }
    for (int k = 0; k < 3; k++) pref[k * (K + 1) + K] = acc[k];
    if (hipMemcpyAsync(sl.d, sl.h, bt_host_bytes(K), hipMemcpyHostToDevice, b->s) != hipSuccess ||
        hipEventRecord(sl.ev, b->s) != hipSuccess) {
        b->err = "batch table upload failed";
        return FIM_E_HIP;
    }
    const long W = acc[1];
    BMap* maps = (BMap*)(sl.d + bt_map_off(K));
    ph.t = (const BMember*)sl.d;
    ph.rows = maps;
    ph.cells = maps + W;
    ph.tiles = maps + 2 * W;
    ph.mem = maps + 3 * W;
    ph.nrows = acc[0];
    ph.ncells = acc[1];
    ph.ntiles = acc[2];
    launch_build_maps((const int*)(sl.d + bt_pref_off(K)), K,
                      std::max(acc[0], std::max(acc[1], acc[2])), (BMap*)ph.rows,
                      (BMap*)ph.cells, (BMap*)ph.tiles, (BMap*)ph.mem, b->s);
    return FIM_OK;
}

// the structure pass of the members' new local systems (one launch per
// kernel for all of them)
static std::vector<BMember> bmembers(const std::vector<fim_model*>& ms) {
    std::vector<BMember> v;
    v.reserve(ms.size());
    for (fim_model* m : ms) v.push_back(bmember(m));
    return v;
}

static fim_status batch_structure(fim_batch* b, const std::vector<fim_model*>& ms) {
    if (ms.empty()) return FIM_OK;
    BPhase ph;
    TRY(batch_upload(b, bmembers(ms), ph));
    launch_structure_seg(ph.t, ph.rows, ph.nrows, ph.mem, ph.K, pc_cell_stride(b->B), b->s);
    return FIM_OK;
}

// the support of the members' converged steps
static fim_status batch_commit(fim_batch* b, const std::vector<fim_model*>& ms) {
    if (ms.empty()) return FIM_OK;
    std::vector<BMember> v = bmembers(ms);
    for (BMember& x : v) x.commit = 1;
    BPhase ph;
    TRY(batch_upload(b, v, ph));
    launch_support_seg(ph.t, ph.cells, ph.ncells, b->s);
    return FIM_OK;
}

static thread_local std::string g_batch_err;

static fim_status batch_check(fim_batch* b, fim_model* const* models, int32_t k, std::string& e) {
    if (!models || k <= 0) { e = "empty batch"; return FIM_E_ARG; }
    int pc_mode = 0;   // fracture-block mode of the members that have blocks
    for (int q = 0; q < k; q++) {
        if (!models[q]) { e = "null model in batch"; return FIM_E_ARG; }
        for (int r = 0; r < q; r++)
            if (models[r] == models[q]) { e = "model listed twice"; return FIM_E_ARG; }
        if (models[q]->B != models[0]->B || models[q]->o.precision != models[0]->o.precision) {
            e = "batch members need the same block size and Krylov precision";
            return FIM_E_ARG;
        }
        if (models[q]->use_pc) {
            const int mode = models[q]->pc_dec ? 2 : 1;
            if (pc_mode && mode != pc_mode) {
                e = "batch members with fracture blocks need the same fracture-block mode";
                return FIM_E_ARG;
            }
            pc_mode = mode;
        }
    }
    (void)b;
    return FIM_OK;
}

fim_status fim_batch_set(fim_batch* b, fim_model* const* models, int32_t k) {
    if (!b) return FIM_E_ARG;
    std::string e;
    fim_status r = batch_check(b, models, k, e);
    if (r != FIM_OK) { b->err = e; return r; }
    fim_model* m = models[0];
    if (k > b->tab.cap) {
        table_free(b->tab);
        TRY(table_alloc(m, b->tab, std::max(k, 2 * b->tab.cap)));
    }
    for (hipEvent_t e2 : b->ev) (void)hipEventDestroy(e2);
    b->ev.assign(k, nullptr);
    for (int q = 0; q < k; q++) HIPX(hipEventCreateWithFlags(&b->ev[q], hipEventDisableTiming));
    b->ms.assign(models, models + k);
    b->B = models[0]->B;
    b->precision = models[0]->o.precision;
    return batch_tables_alloc(b);
}

fim_status fim_batch_create(fim_model* const* models, int32_t k, void* hip_stream, fim_batch** out) {
    if (!out) return FIM_E_ARG;
    *out = nullptr;
    std::string e;
    fim_status r = batch_check(nullptr, models, k, e);
    if (r != FIM_OK) { g_batch_err = e; return r; }
    fim_batch* b = new fim_batch();
    if (hip_stream) {
        b->s = (hipStream_t)hip_stream;
    } else if (hipStreamCreate(&b->s) != hipSuccess) {
        g_batch_err = "hipStreamCreate failed";
        delete b;
        return FIM_E_HIP;
    } else {
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming) != hipSuccess) {
        g_batch_err = "hipEventCreate failed";
        (void)fim_batch_destroy(b);
        return FIM_E_HIP;
    }
    r = fim_batch_set(b, models, k);
    if (r != FIM_OK) {
        g_batch_err = b->err.empty() ? models[0]->err : b->err;
        (void)fim_batch_destroy(b);
        return r;
    }
    *out = b;
    return FIM_OK;
}

fim_status fim_batch_destroy(fim_batch* b) {
    if (!b) return FIM_E_ARG;
    if (b->s) (void)hipStreamSynchronize(b->s);
    table_free(b->tab);
    batch_tables_free(b);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    if (b->done_ev) (void)hipEventDestroy(b->done_ev);
    if (b->own_stream && b->s) (void)hipStreamDestroy(b->s);
    delete b;
    return FIM_OK;
}

const char* fim_batch_last_error(const fim_batch* b) {
    return b ? b->err.c_str() : g_batch_err.c_str();
}

// One Newton iteration of every member (Algorithm 1, full Newton or the
// residual-based mode) on the batch stream, one launch per kernel for all
// members: the timestep starts (and one synchronisation for their n_A),
// assembly and scaling, one batched Krylov solve, the updates, the sets and
// compaction, one synchronisation for the status words, then the supports
// of the converged steps and the structure of the next local systems.
fim_status fim_batch_newton_step(fim_batch* b, const double* dts, const int32_t* modes,
                                 fim_iter_stats* stats, int32_t* codes) {
    if (!b || !dts || !modes || !codes) return FIM_E_ARG;
    const int K = (int)b->ms.size();
    auto is_dd = [&](int q) { return modes[q] == FIM_DD || modes[q] == FIM_DD_ADD; };
    for (int q = 0; q < K; q++) {
        if (modes[q] < FIM_FULL || modes[q] > FIM_DD_ADD) {
            b->err = "batched steps run FIM_FULL, FIM_LOCAL, FIM_DD, FIM_RESID or FIM_DD_ADD";
            return FIM_E_ARG;
        }
        if (!(dts[q] > 0.0) || !std::isfinite(dts[q])) {
            b->err = "dt must be positive";
            return FIM_E_ARG;
        }
    }
    std::vector<hipStream_t> saved(K);
    // hand the members over to the batch stream
    for (int q = 0; q < K; q++) {
        fim_model* m = b->ms[q];
        saved[q] = m->s;
        if (m->s != b->s) {
            if (hipEventRecord(b->ev[q], m->s) != hipSuccess ||
                hipStreamWaitEvent(b->s, b->ev[q], 0) != hipSuccess) {
                b->err = "stream hand-over failed";
                return FIM_E_HIP;
            }
        }
        m->s = b->s;
        if (stats) std::memset(&stats[q], 0, sizeof(fim_iter_stats));
        codes[q] = FIM_OK;
    }
    auto restore = [&]() {
        (void)hipEventRecord(b->done_ev, b->s);
        for (int q = 0; q < K; q++) {
            b->ms[q]->s = saved[q];
            if (saved[q] != b->s) (void)hipStreamWaitEvent(saved[q], b->done_ev, 0);
        }
    };
    // Algorithm 2 members: one inner iteration each with their own
    // launches (a subdomain solve or an additive sweep has its own
    // host-driven phase machine), on the batch stream
    for (int q = 0; q < K; q++)
        if (is_dd(q))
            codes[q] = fim_newton_step(b->ms[q], dts[q], modes[q], stats ? &stats[q] : nullptr);
    // members that start a timestep: u^n, accumulation and the first
    // active set in one launch per kernel, one synchronisation for the new
    // n_A, then one structure pass
    std::vector<fim_model*> starters, pending;
    std::vector<BMember> bent;
    for (int q = 0; q < K; q++) {
        fim_model* m = b->ms[q];
        if (is_dd(q)) continue;
        if (m->in_step && (dts[q] != m->step_dt || modes[q] != m->step_mode)) {
            m->err = "dt or mode changed inside a timestep";
            codes[q] = FIM_E_STATE;
            continue;
        }
        if (!m->in_step) {
            const int kind = begin_state(m, dts[q], modes[q]);
            BMember x = bmember(m);
            x.begin = kind;
            x.compact = kind <= 3 ? 1 : 0;
            x.layers = kind == 2 ? std::min(m->o.m_layers, MAX_LAYERS) : 0;
            bent.push_back(x);
            starters.push_back(m);
            if (kind <= 3) pending.push_back(m);
        }
    }
    if (!starters.empty()) {
        fim_model* lead = starters[0];
        BPhase ph;
        fim_status r = batch_upload(b, bent, ph);
        if (r != FIM_OK) {
            restore();
            return r;
        }
        const int pi = pbeg(lead, PK_SETUP);
        launch_begin_seg(b->B, ph.t, ph.cells, ph.ncells, ph.layers, b->s);
        for (fim_model* m : starters)
            if (m->step_mode == FIM_LOCAL) frac_closure(m);
        launch_compact_seg(ph.t, ph.tiles, ph.ntiles, b->s);
        pend(lead, pi, ph.ncells * NT);
        if (!pending.empty()) {
            launch_status_seg(ph.t, ph.mem, ph.K, b->dstat, b->s);
            if (hipStreamSynchronize(b->s) != hipSuccess) {
                b->err = "hipStreamSynchronize failed";
                restore();
                return FIM_E_HIP;
            }
            for (size_t t = 0; t < starters.size(); t++) {
                pflush(starters[t]);
                if (bent[t].compact) starters[t]->nA = b->hstat[t].dint[1];
            }
            r = batch_structure(b, pending);
            if (r != FIM_OK) {
                restore();
                return r;
            }
            for (fim_model* m : pending)
                if (m->step_mode == FIM_FULL || m->step_mode == FIM_RESID) {
                    m->full_ready = true;
                    m->nA = m->n;
                }
        }
    }
    // the live members: one launch per kernel for all of them
    std::vector<fim_model*> live;
    std::vector<int> pos;
    for (int q = 0; q < K; q++) {
        if (codes[q] != FIM_OK || is_dd(q)) continue;
        fim_model* m = b->ms[q];
        if (m->nA == 0) {
            codes[q] = empty_iteration(m, stats ? &stats[q] : nullptr);
            continue;
        }
        live.push_back(m);
        pos.push_back(q);
    }
    if (!live.empty()) {
        fim_model* lead = live[0];
        BPhase ph;
        fim_status r = batch_upload(b, bmembers(live), ph);
        if (r != FIM_OK) {
            restore();
            return r;
        }
        int pi = pbeg(lead, PK_ASSEMBLE);
        launch_assemble_seg(b->B, ph.t, ph.rows, ph.nrows, b->s);
        pend(lead, pi, ph.nrows * NT);
        pi = pbeg(lead, PK_PRECOND);
        launch_precond_seg(b->B, b->precision == FIM_MIXED, ph.t, ph.rows, ph.nrows, b->s);
        pend(lead, pi, ph.nrows * NT);
        r = solve_batch(live, b->tab, b->s, true);
        if (r != FIM_OK) {
            b->err = live[0]->err;
            restore();
            return r;
        }
        pi = pbeg(lead, PK_UPDATE);
        launch_update_seg(b->B, ph.t, ph.rows, ph.nrows, ph.mem, ph.K, b->s);
        pend(lead, pi, ph.nrows * NT);
        for (size_t t = 0; t < live.size(); t++) {
            newton_classes(live[t]);
            newton_update_stats(live[t], stats ? &stats[pos[t]] : nullptr);
        }
        pi = pbeg(lead, PK_SETS);
        launch_sets_seg(b->B, ph.t, ph.rows, ph.nrows, ph.cells, ph.ncells, ph.mem, ph.K,
                        ph.layers, ph.any_resid, b->s);
        for (fim_model* m : live)
            if (m->step_mode == FIM_LOCAL) frac_closure(m);
        launch_compact_seg(ph.t, ph.tiles, ph.ntiles, b->s);
        pend(lead, pi, ph.ncells * NT);
        launch_status_seg(ph.t, ph.mem, ph.K, b->dstat, b->s);
        for (fim_model* m : live)
            if (m->step_mode == FIM_RESID) m->full_ready = false;   // l2g / g2l: the new set
        if (hipStreamSynchronize(b->s) != hipSuccess) {
            b->err = "hipStreamSynchronize failed";
            restore();
            return FIM_E_HIP;
        }
        std::vector<fim_model*> next, done;
        for (size_t t = 0; t < live.size(); t++) {
            fim_model* m = live[t];
            pflush(m);
            *m->hns = b->hstat[t].ns;
            for (int k = 0; k < 4; k++) m->hint[k] = b->hstat[t].dint[k];
            BatchDefer d;
            codes[pos[t]] = newton_post_finish(m, stats ? &stats[pos[t]] : nullptr, &d);
            if (d.structure) next.push_back(m);
            if (d.commit) done.push_back(m);
        }
        r = batch_commit(b, done);
        if (r == FIM_OK) r = batch_structure(b, next);
        if (r != FIM_OK) {
            restore();
            return r;
        }
    }
    restore();
    return FIM_OK;
}

// ------------------------------------------------------- cell classes
fim_status fim_flags_enable(fim_model* m, int32_t on) {
    if (!m) return FIM_E_ARG;
    if (on && !m->classes) {
        TRY(dal(m, &m->classes, (size_t)m->n));
        launch_fill_u8(m->classes, m->n, 0, m->s);
    }
    m->flags_on = on != 0;
    return FIM_OK;
}

fim_status fim_get_flags(fim_model* m, uint8_t* out) {
    if (!m || !out) return FIM_E_ARG;
    if (!m->classes) {
        m->err = "cell classes are not recorded (fim_flags_enable)";
        return FIM_E_STATE;
    }
    HIPX(hipMemcpyAsync(out, m->classes, m->n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

// ----------------------------------------------------------- profiling
fim_status fim_profile_enable(fim_model* m, int32_t on) {
    if (!m) return FIM_E_ARG;
    HIPX(hipStreamSynchronize(m->s));
    pflush(m);
    m->prof.on = on != 0;
    for (int k = 0; k < PK_N; k++) {
        m->prof.ms[k] = 0.0;
        m->prof.rows[k] = 0.0;
        m->prof.nnzb[k] = 0.0;
        m->prof.aux[k] = 0.0;
        m->prof.cnt[k] = 0;
    }
    return FIM_OK;
}

int32_t fim_profile_read(fim_model* m, fim_kernel_profile* out, int32_t cap) {
    if (!m) return 0;
    if (hipStreamSynchronize(m->s) == hipSuccess) pflush(m);
    int k = 0;
    for (; k < PK_N && k < cap; k++) {
        std::memset(out[k].name, 0, sizeof(out[k].name));
        std::strncpy(out[k].name, kPkName[k], sizeof(out[k].name) - 1);
        out[k].launches = m->prof.cnt[k];
        out[k].total_ms = m->prof.ms[k];
        out[k].rows = m->prof.rows[k];
        out[k].nnzb = m->prof.nnzb[k];
        out[k].aux = m->prof.aux[k];
    }
    return k;
}

// --------------------------------------------------------- inspection
fim_status fim_inspect_assemble(fim_model* m, const double* u_old, const double* u_iter,
                                const int8_t* status, double dt, const uint8_t* act,
                                int32_t* n_active, int32_t* l2g, double* F,
                                int32_t* row_ptr, int32_t* col, double* val,
                                int64_t cap_blocks) {
    if (!m || !u_old || !u_iter || !n_active || !F || !row_ptr || !col || !val || !(dt > 0))
        return FIM_E_ARG;
    const size_t nb = (size_t)m->n * m->B;
    m->in_step = false;
    m->full_ready = false;
    HIPX(hipMemcpyAsync(m->un, u_old, nb * sizeof(double), hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->u, u_iter, nb * sizeof(double), hipMemcpyHostToDevice, m->s));
    if (status) {
        HIPX(hipMemcpyAsync(m->st, status, m->n, hipMemcpyHostToDevice, m->s));
        HIPX(hipMemcpyAsync(m->stn, status, m->n, hipMemcpyHostToDevice, m->s));
    } else {
        launch_fill_u8((uint8_t*)m->st, m->n, 0, m->s);
        launch_fill_u8((uint8_t*)m->stn, m->n, 0, m->s);
    }
    launch_accumulation(m->fk, m->n, m->un, m->stn, m->g, m->f, m->Mn, m->s);
    if (act) HIPX(hipMemcpyAsync(m->act, act, m->n, hipMemcpyHostToDevice, m->s));
    else launch_fill_u8(m->act, m->n, 1, m->s);
    TRY(prepare_active(m, false));
    m->step_dt = dt;
    const LocalSys ls = lsys(m);
    launch_assemble(m->fk, m->nA, ls, m->g, m->f, m->u, m->st, m->Mn, 1.0 / dt, m->s);
    const int nA = m->nA, B = m->B, BB = B * B;
    const int nsl = (nA + SLICE - 1) / SLICE;
    std::vector<int> swidth(nsl), hl2g(nA);
    HIPX(hipMemcpyAsync(swidth.data(), m->swidth, nsl * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    const long slots = (long)nsl * SLICE * ls.wcap;
    std::vector<int> hcol(slots);
    std::vector<double> hJ(slots * BB);
    HIPX(hipMemcpyAsync(hl2g.data(), m->l2g, nA * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(hcol.data(), m->col, slots * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(hJ.data(), m->J, slots * BB * sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(F, m->F, (size_t)nA * B * sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    *n_active = nA;
    if (l2g) std::memcpy(l2g, hl2g.data(), nA * sizeof(int));
    long nz = 0;
    row_ptr[0] = 0;
    for (int r = 0; r < nA; r++) {
        const int w = swidth[r / SLICE];
        for (int k = 0; k < w; k++) {
            const long pos = slot_of(ls, r, k);
            if (k > 0 && hcol[pos] == r) break;   // padding
            if (nz >= cap_blocks) {
                m->err = "cap_blocks too small";
                return FIM_E_ARG;
            }
            col[nz] = hcol[pos];
            std::memcpy(val + nz * BB, hJ.data() + pos * BB, BB * sizeof(double));
            nz++;
        }
        row_ptr[r + 1] = (int32_t)nz;
    }
    m->inspect_ready = true;
    return FIM_OK;
}

fim_status fim_inspect_solve(fim_model* m, double* x, int32_t* iters, double* relres) {
    if (!m || !x) return FIM_E_ARG;
    if (!m->inspect_ready) {
        m->err = "call fim_inspect_assemble first";
        return FIM_E_STATE;
    }
    TRY(linear_solve(m));
    HIPX(hipMemcpyAsync(x, m->x64, (size_t)m->nA * m->B * sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    if (iters) *iters = m->last_kry;
    if (relres) *relres = m->last_relres;
    return FIM_OK;
}

fim_status fim_inspect_sets(fim_model* m, const uint8_t* act_in, const double* dp_abs,
                            double eps, int32_t layers, uint8_t* act_out, uint8_t* bnd_out,
                            int32_t* l2g_out, int32_t* n_active, int32_t* is_expand) {
    if (!m || !act_in || !dp_abs || !act_out || !bnd_out || !l2g_out || !n_active || !is_expand)
        return FIM_E_ARG;
    if (layers < 0 || layers > MAX_LAYERS) {
        m->err = "layers must be in [0, 8]";
        return FIM_E_ARG;
    }
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    HIPX(hipMemcpyAsync(m->act, act_in, m->n, hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->dp_abs, dp_abs, m->n * sizeof(double), hipMemcpyHostToDevice, m->s));
    TRY(prepare_active(m, true));
    launch_fill_i32(m->dint, 1, 0, m->s);
    launch_mark_expand(m->nA, m->l2g, m->bnd, m->dp_abs, eps, layers, m->g, m->act, nullptr,
                       m->dint, m->lvl, m->s);
    launch_shrink(m->nA, m->l2g, m->dp_abs, eps, m->g, m->act, m->dint, m->s);
    frac_closure(m);
    TRY(read_int(m));
    *is_expand = m->hint[0] != 0;
    TRY(prepare_active(m, true));
    HIPX(hipMemcpyAsync(act_out, m->act, m->n, hipMemcpyDeviceToHost, m->s));
    // boundary flags are meaningful on active cells only: export 0 elsewhere
    std::vector<uint8_t> hb(m->n);
    HIPX(hipMemcpyAsync(hb.data(), m->bnd, m->n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(l2g_out, m->l2g, m->nA * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    for (int i = 0; i < m->n; i++) bnd_out[i] = act_out[i] ? hb[i] : 0;
    *n_active = m->nA;
    return FIM_OK;
}

fim_status fim_inspect_resid_error(fim_model* m, const double* u_old, const double* u_iter,
                                   const int8_t* status, double dt, double* err_out) {
    if (!m || !u_old || !u_iter || !err_out || !(dt > 0.0) || !std::isfinite(dt))
        return FIM_E_ARG;
    const size_t nb = (size_t)m->n * m->B;
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    HIPX(hipMemcpyAsync(m->un, u_old, nb * sizeof(double), hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->u, u_iter, nb * sizeof(double), hipMemcpyHostToDevice, m->s));
    if (status) {
        HIPX(hipMemcpyAsync(m->st, status, m->n, hipMemcpyHostToDevice, m->s));
        HIPX(hipMemcpyAsync(m->stn, status, m->n, hipMemcpyHostToDevice, m->s));
    } else {
        launch_fill_u8((uint8_t*)m->st, m->n, 0, m->s);
        launch_fill_u8((uint8_t*)m->stn, m->n, 0, m->s);
    }
    launch_accumulation(m->fk, m->n, m->un, m->stn, m->g, m->f, m->Mn, m->s);
    launch_resid_err(m->fk, m->n, m->g, m->f, m->u, m->st, m->Mn, dt, m->last_dp, m->s);
    HIPX(hipMemcpyAsync(err_out, m->last_dp, m->n * sizeof(double), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

fim_status fim_inspect_resid_sets(fim_model* m, const double* err, double tol, int32_t layers,
                                  uint8_t* act_out, int32_t* l2g_out, int32_t* n_active,
                                  int32_t* n_unconverged) {
    if (!m || !err || !act_out || !l2g_out || !n_active || !n_unconverged) return FIM_E_ARG;
    if (layers < 0 || layers > MAX_LAYERS) {
        m->err = "layers must be in [0, 8]";
        return FIM_E_ARG;
    }
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    HIPX(hipMemcpyAsync(m->last_dp, err, m->n * sizeof(double), hipMemcpyHostToDevice, m->s));
    launch_fill_i32(m->dint, 1, 0, m->s);
    launch_mark_resid(m->n, m->last_dp, tol, layers, m->g, m->act, m->dint, m->lvl, m->s);
    compact(m);
    TRY(read_int(m));
    m->nA = m->hint[1];
    *n_unconverged = m->hint[0];
    *n_active = m->nA;
    HIPX(hipMemcpyAsync(act_out, m->act, m->n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(l2g_out, m->l2g, m->nA * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    return FIM_OK;
}

fim_status fim_inspect_pc_blocks(fim_model* m, const uint8_t* act, int32_t* n_active,
                                 int32_t* l2g, int32_t* blk_start, int32_t* blk_rows) {
    if (!m || !n_active || !l2g || !blk_start || !blk_rows) return FIM_E_ARG;
    if (!m->use_pc) {
        m->err = "the model has no fracture blocks";
        return FIM_E_STATE;
    }
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    if (act) HIPX(hipMemcpyAsync(m->act, act, m->n, hipMemcpyHostToDevice, m->s));
    else launch_fill_u8(m->act, m->n, 1, m->s);
    TRY(prepare_active(m, false));
    const int nA = m->nA;
    std::vector<int> info(nA);
    HIPX(hipMemcpyAsync(l2g, m->l2g, nA * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(info.data(), m->pcinfo, nA * sizeof(int), hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    *n_active = nA;
    for (int r = 0; r < nA; r++) {
        blk_start[r] = (r / KB_NT) * KB_NT + (info[r] >> 16);
        blk_rows[r] = info[r] & 0xffff;
    }
    return FIM_OK;
}

// Algorithm 2 phase-1 set logic (Section 4.4, Step 1) on given inputs.
fim_status fim_inspect_dd_expand(fim_model* m, const uint8_t* vt_in, const uint8_t* act_in,
                                 const uint8_t* bnd_in, const double* dp_abs, double eps,
                                 int32_t layers, uint8_t* vt_out, uint8_t* act_out,
                                 uint8_t* bnd_out, uint8_t* outer_out, int32_t* n_active,
                                 int32_t* is_expand) {
    if (!m || !vt_in || !act_in || !bnd_in || !dp_abs || !vt_out || !act_out || !bnd_out ||
        !outer_out || !n_active || !is_expand)
        return FIM_E_ARG;
    if (layers < 0 || layers > MAX_LAYERS) {
        m->err = "layers must be in [0, 8]";
        return FIM_E_ARG;
    }
    const int n = m->n;
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    m->dd_valid = false;
    HIPX(hipMemcpyAsync(m->act, act_in, n, hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->vt, vt_in, n, hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->bnd, bnd_in, n, hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->dp_abs, dp_abs, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                        m->s));
    TRY(prepare_active(m, false));
    bool expand = false;
    TRY(dd_expand_sets(m, eps, layers, &expand));
    std::vector<uint8_t> hb(n), ho(n);
    HIPX(hipMemcpyAsync(vt_out, m->vt, n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(act_out, m->act, n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(hb.data(), m->bnd, n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipMemcpyAsync(ho.data(), m->outer, n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    *is_expand = expand ? 1 : 0;
    if (!expand) {
        // no subdomain follows: the next sets are empty
        std::memset(act_out, 0, n);
        std::memset(bnd_out, 0, n);
        std::memset(outer_out, 0, n);
        *n_active = 0;
        return FIM_OK;
    }
    for (int i = 0; i < n; i++) {
        bnd_out[i] = act_out[i] ? hb[i] : 0;
        outer_out[i] = ho[i];
    }
    *n_active = m->nA;
    return FIM_OK;
}

// Algorithm 2 phase-2 subdomain choice (Section 4.4, Step 2) on given
// subdomain lists and latest updates.
fim_status fim_inspect_dd_pick(fim_model* m, int32_t n_sub, const int32_t* cells_ptr,
                               const int32_t* cells, const int32_t* outer_ptr,
                               const int32_t* outer, const double* last_dp, double eps,
                               int32_t next, double* sub_max, int32_t* pick,
                               int32_t* new_sweep) {
    if (!m || !cells_ptr || !outer_ptr || !last_dp || !sub_max || !pick || !new_sweep)
        return FIM_E_ARG;
    if (n_sub < 1 || n_sub > MAX_SUBS || next < 0 || next > n_sub) {
        m->err = "n_sub must be in [1, 64] and next in [0, n_sub]";
        return FIM_E_ARG;
    }
    const int n = m->n;
    for (const int32_t* ptr : {cells_ptr, outer_ptr}) {
        if (ptr[0] != 0) {
            m->err = "list offsets must start at 0";
            return FIM_E_ARG;
        }
        for (int k = 0; k < n_sub; k++)
            if (ptr[k + 1] < ptr[k]) {
                m->err = "list offsets must not decrease";
                return FIM_E_ARG;
            }
    }
    const long nc = cells_ptr[n_sub], no = outer_ptr[n_sub];
    if ((nc > 0 && !cells) || (no > 0 && !outer)) return FIM_E_ARG;
    for (long q = 0; q < nc; q++)
        if (cells[q] < 0 || cells[q] >= n) {
            m->err = "cell index out of range";
            return FIM_E_ARG;
        }
    for (long q = 0; q < no; q++)
        if (outer[q] < 0 || outer[q] >= n) {
            m->err = "cell index out of range";
            return FIM_E_ARG;
        }
    m->in_step = false;
    m->full_ready = false;
    m->inspect_ready = false;
    m->dd_valid = false;
    m->subs.clear();
    m->sd_used = m->ob_used = 0;
    TRY(dd_grow(m, &m->sd_cells, &m->sd_cap, nc + 1));
    TRY(dd_grow(m, &m->sd_outer, &m->ob_cap, no + 1));
    if (nc > 0)
        HIPX(hipMemcpyAsync(m->sd_cells, cells, nc * sizeof(int), hipMemcpyHostToDevice, m->s));
    if (no > 0)
        HIPX(hipMemcpyAsync(m->sd_outer, outer, no * sizeof(int), hipMemcpyHostToDevice, m->s));
    HIPX(hipMemcpyAsync(m->last_dp, last_dp, (size_t)n * sizeof(double), hipMemcpyHostToDevice,
                        m->s));
    std::vector<DDSub> subs(n_sub);
    for (int k = 0; k < n_sub; k++) {
        subs[k].cells_off = cells_ptr[k];
        subs[k].cells_n = cells_ptr[k + 1] - cells_ptr[k];
        subs[k].outer_off = outer_ptr[k];
        subs[k].outer_n = outer_ptr[k + 1] - outer_ptr[k];
    }
    launch_sub_max(n_sub, subs.data(), m->sd_cells, m->sd_outer, m->last_dp, m->dsub, m->s);
    TRY(sync_read(m, m->hsub, m->dsub, n_sub * sizeof(double)));
    std::memcpy(sub_max, m->hsub, n_sub * sizeof(double));
    bool ns = false;
    *pick = dd_pick(m->hsub, n_sub, eps, next, &ns);
    *new_sweep = ns ? 1 : 0;
    return FIM_OK;
}

fim_status fim_get_dd_total(fim_model* m, uint8_t* vt_out, int32_t* n_sub) {
    if (!m || !vt_out || !n_sub) return FIM_E_ARG;
    if (!m->dd_valid) {
        m->err = "no Algorithm 2 timestep has run since the last inspection call";
        return FIM_E_STATE;
    }
    HIPX(hipMemcpyAsync(vt_out, m->vt, m->n, hipMemcpyDeviceToHost, m->s));
    HIPX(hipStreamSynchronize(m->s));
    *n_sub = (int32_t)m->subs.size();
    return FIM_OK;
}

} // extern "C"
