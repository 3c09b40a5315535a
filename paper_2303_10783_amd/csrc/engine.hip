// Host side of the solidification step library: argument validation, device
// memory, the time-step driver of Algorithm 1, the Krylov orchestration and
// the C ABI declared in sol.h.
//
// Krylov orchestration: convergence is decided on the device (every
// workgroup of an iteration kernel totals the partial sums of the previous
// kernel and takes the same decision; workgroup 0 records it in
// KState::status; every kernel of a solve that is no longer RUNNING returns
// at once).  The host queues
// iterations in chunks and reads the status array through one lagging
// event: while it inspects chunk k the device already runs chunk k+1, so the
// GPU never waits for the host; the price is at most one chunk of no-op
// launches after convergence.  Chunk sizes follow the iteration count of the
// same solve in the previous step.
#include "sol.h"
#include "sol_dev.hpp"
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace sol;

static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SOL_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define RCHK(expr)                  \
    do {                            \
        int r_ = (expr);            \
        if (r_ != SOL_OK) return r_; \
    } while (0)

// ------------------------------------------------------------------ memory

// Device memory of a case: one slab of the case's whole footprint, handed
// out in 256-byte aligned pieces (one allocator call per case instead of
// about a hundred; with torch's allocator each call crosses into Python).
// A request beyond the slab gets an allocation of its own.
struct Mem {
    sol_device_ctx ctx{};
    bool has_ctx = false;
    std::vector<void *> blocks;
    size_t bytes = 0;
    char *slab = nullptr;
    size_t slab_size = 0, slab_used = 0;
    void *raw(size_t n)
    {
        void *p = nullptr;
        if (has_ctx) p = ctx.alloc(n, ctx.user);
        else if (hipMalloc(&p, n) != hipSuccess) p = nullptr;
        if (p) { blocks.push_back(p); bytes += n; }
        return p;
    }
    void reserve(size_t n)
    {
        n = (n + 255) & ~size_t(255);
        slab = (char *)raw(n);
        slab_size = slab ? n : 0;
        slab_used = 0;
    }
    void *get(size_t n)
    {
        n = (std::max<size_t>(n, 256) + 255) & ~size_t(255);
        if (slab && slab_used + n <= slab_size) {
            void *p = slab + slab_used;
            slab_used += n;
            return p;
        }
        return raw(n);
    }
    void release()
    {
        for (void *p : blocks) {
            if (has_ctx) ctx.free(p, ctx.user);
            else (void)hipFree(p);
        }
        blocks.clear();
        bytes = 0;
        slab = nullptr;
        slab_size = slab_used = 0;
    }
};

// ------------------------------------------------------------------ sizes

struct Sizes {
    int dim, nx, ny, nz, ncell, nd, maxn, ntile_cell;
    int nsys[NSYS], sdim[NSYS][3];
};

static void compute_sizes(const sol_grid &g, Sizes &z)
{
    z.dim = g.dim;
    z.nx = g.nx;
    z.ny = g.ny;
    z.nz = g.dim == 3 ? g.nz : 1;
    z.ncell = z.nx * z.ny * z.nz;
    z.nd = 2 * z.dim + 1;
    z.maxn = 0;
    for (int s = 0; s < NSYS; ++s) {
        int d[3] = {z.nx, z.ny, z.nz};
        if (s <= SW) d[s] -= 1;
        if (s == SW && z.dim != 3) d[0] = d[1] = d[2] = 0;
        for (int a = 0; a < 3; ++a) { if (d[a] < 0) d[a] = 0; z.sdim[s][a] = d[a]; }
        z.nsys[s] = d[0] * d[1] * d[2];
        z.maxn = std::max(z.maxn, z.nsys[s]);
    }
    z.ntile_cell = ceil_div(z.ncell, TILE);
}

// multigrid levels of the pressure grid: every count above 1 halves
// (rounding up) from one level to the next, down to nglob, the first level
// >= 1 with at most MG_EXACT_MAX cells (MG_EXACT_MAX_LARGE for grids of at
// least MG_LARGE_CELLS cells), solved exactly
struct MGDims {
    int nlev = 0, nglob = 0;
    int nbig = 0;                 // large grids: the first level >= 1 with <= MG_EXACT_MAX_LARGE cells, if above nglob
    int d[MG_MAXLEV][3];
    int n[MG_MAXLEV];
};

static void mg_dims(const Sizes &z, MGDims &m)
{
    int d0 = z.nx, d1 = z.ny, d2 = z.nz;
    const bool large = (int64_t)d0 * d1 * d2 >= MG_LARGE_CELLS;
    for (;;) {
        const int l = m.nlev++;
        m.d[l][0] = d0;
        m.d[l][1] = d1;
        m.d[l][2] = d2;
        m.n[l] = d0 * d1 * d2;
        if (large && l >= 1 && m.nbig == 0 && m.n[l] <= MG_EXACT_MAX_LARGE) m.nbig = l;
        if (l >= 1 && m.n[l] <= MG_EXACT_MAX) {
            m.nglob = l;
            break;
        }
        if (m.nlev == MG_MAXLEV) break;
        d0 = (d0 + 1) / 2;
        d1 = (d1 + 1) / 2;
        d2 = (d2 + 1) / 2;
    }
    if (m.nglob == 0) m.nglob = m.nlev - 1;
    if (m.nbig >= m.nglob) m.nbig = 0;
}

// Krylov work vectors per set: r, rh, p0, p1, v0, v1, t, r1 (FP64); the FP32
// sets add the inner solution and right-hand side (7, 8) and r1 (9)
constexpr int NWORK = 8, NWORK32 = 10;

// total device bytes of one case (matches the allocations in sol_create)
static size_t footprint(const Sizes &z, int precision)
{
    auto al = [](size_t n) { return (std::max<size_t>(n, 256) + 255) & ~size_t(255); };
    size_t b = 0;
    const size_t D = sizeof(double), F = sizeof(float);
    size_t nf = 0;
    for (int s = 0; s < 3; ++s) nf += std::max(z.nsys[s], 1);
    b += 5 * (al(nf * D));                                       // u,v,w / us / un / 2 history of us
    b += 13 * al((size_t)z.ncell * D);                          // p T C gl Cl Cs phi Cnew Tstar, 4 history
    for (int s = 0; s < NSYS; ++s) {
        const size_t n = std::max(z.nsys[s], 1);
        b += al(z.nd * n * D) + 2 * al(n * D);                   // A, b, minv
        if (s != SP && s != SC) b += al(z.nd * n * D);           // constant parts
        if (precision) b += al(z.nd * n * F) + al(n * F);
    }
    b += 3 * NWORK * al((size_t)z.maxn * D);                    // Krylov work vectors
    if (precision) b += 3 * NWORK32 * al((size_t)z.maxn * F);   // FP32 inner work vectors
    b += al((size_t)z.ntile_cell * 4 * D) + 2 * al(256);         // reductions, counters, step
    {
        MGDims m;                                                // pressure multigrid hierarchy
        mg_dims(z, m);
        for (int l = 1; l < m.nlev; ++l) {
            b += 4 * al((size_t)m.n[l] * D);                     // inverse diagonal, rhs, correction, pre-smoothed
            if (precision) b += 4 * al((size_t)m.n[l] * F);
        }
        if (z.dim == 2) {                                        // level 0 pre-smoothed
            b += al((size_t)m.n[0] * D);
            if (precision) b += al((size_t)m.n[0] * F);
        }
        const size_t nx2 = (size_t)m.n[m.nglob] * m.n[m.nglob];  // dense inverse of the exact level
        b += al(nx2 * D) + al(nx2 * F);
        b += al(mg_gj_work(m.n[m.nglob]) * D);                   // its elimination scratch
        if (m.nbig) {                                            // large grids alone: a larger exact level
            const size_t nb2 = (size_t)m.n[m.nbig] * m.n[m.nbig];
            b += al(nb2 * D) + al(nb2 * F) + al(mg_gj_work(m.n[m.nbig]) * D);
        }
        b += al(sizeof(MLevel) * MG_MAXLEV) * (precision ? 2 : 1);
    }
    return b;
}

// Rows per tile of a solve.  Default: 1..8 rows per thread, aiming at
// <= ~384 tiles (<= ~192 below MG_LARGE_CELLS rows) so that the per-kernel
// totals of the partial sums stay cheap.  sol_autotune replaces the default for a size class (stencil
// width, floor(log2 n)) by the fastest measured choice; the table is
// process-wide so a case gets the same tiles alone and in a batch.
static std::mutex g_tune_mu;
static std::map<int, int> g_tuned_rpt;

static int size_class(int n, int nd) { return nd * 64 + (n > 0 ? 31 - __builtin_clz((unsigned)n) : 0); }

// multigrid: level-1 cells per tile of the level-0 kernels (1..8 per
// thread, aiming at <= ~1024 tiles); tuned per size class like the above
static std::map<int, int> g_tuned_cpt;

static int mg_cells_per_tile(int n, int nd, int cn)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned_cpt.find(size_class(n, nd));
        if (it != g_tuned_cpt.end()) return it->second;
    }
    return TILE * std::max(1, std::min(8, ceil_div(cn, TILE * 1024)));
}

static int rows_per_tile(int n, int nd)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned_rpt.find(size_class(n, nd));
        if (it != g_tuned_rpt.end()) return it->second;
    }
    // below MG_LARGE_CELLS rows (the sizes that run in batches) ~192 tiles:
    // fewer, larger workgroups per case gave the 64-cavity batch 256 -> 293 M
    // cell-updates/s (FP64) and 374 -> 399 M (mixed); 500x300 stepped alone
    // is 1 % faster with ~384
    const int per = n < MG_LARGE_CELLS ? 192 : 384;
    const int m = std::max(1, std::min(8, ceil_div(n, TILE * per)));
    return TILE * m;
}

// ------------------------------------------------------------------ timing

struct JobSet;
struct TSample { int cls; int64_t iter; const JobSet *set; int tsize; hipEvent_t a, b; int count = 1; bool two = false; bool s1 = false;
                 bool fwd = false; };
struct TAcc { int64_t n = 0; double ms = 0.0, bytes = 0.0; };

// algorithmic bytes per row of one launch: matrix values and every vector
// element read or written once; tsize = bytes per value (8 FP64, 4 FP32);
// fwd: the forward assembly route, which reads the stored constant part (the
// stencil route forms it in registers)
static double row_bytes(int cls, int nd, int dim, int tsize, bool fwd = false)
{
    switch (cls) {
    case SOL_KCLASS_CG: return (nd + 11.0) * tsize;     // A, r, w, s, M, p, x; p, s, x, r, w
    case SOL_KCLASS_BICG_A: return (nd + 11.0) * tsize; // A, r, v, t, p, M, rh, x; x, r', p', v'
    case SOL_KCLASS_BICG_B: return (nd + 5.0) * tsize;  // A, r, v, M, rh; t
    // multigrid (the pressure operator and its Jacobi inverse diagonal are
    // applied from their closed forms, no matrix values are read)
    case SOL_KCLASS_MG_PQ: return 4.0 * tsize;           // z, p_old; p, q
    case SOL_KCLASS_MG_DOWN0:                            // r, q, x, p; x, r; level-1 rhs (2D: and x2)
        return (6.0 + (dim == 2) + 1.0 / (1 << dim)) * tsize;
    case SOL_KCLASS_MG_UP0:                              // r, level-1 correction (2D: and x2); z
        return (2.0 + (dim == 2) + 1.0 / (1 << dim)) * tsize;
    case SOL_KCLASS_MG_COARSE: return 0.0;
    case SOL_KCLASS_ASM_MOM: return (fwd ? 16.0 : 8.0) * nd + 8.0 * dim + 48.0;
    case SOL_KCLASS_ASM_TRN: return (fwd ? 24.0 : 16.0) * nd + 8.0 * dim + 56.0;
    case SOL_KCLASS_PHASE: return 96.0 + 16.0 * dim;
    }
    return 0.0;
}

// A BiCGSTAB A launch that ended its solve at the half step (x += alpha M p):
// x, p, M; x (two sweeps: and the nd - 1 off-diagonals of A)
static double half_exit_bytes(int nd, bool two, int tsize) { return (two ? nd + 3.0 : 4.0) * tsize; }

// A BiCGSTAB B launch that stages the solve in LDS at FP64 forms M from the
// diagonal of A and reads no M: one value per row fewer
static bool b_without_m(const TSample &s, const KJob &J, int nd)
{
    return s.cls == SOL_KCLASS_BICG_B && s.tsize == 8 && (nd == 7 ? s.s1 : J.staged != 0);
}

// ------------------------------------------------------------------ handle

struct Group;

struct sol_handle {
    sol_grid grid{};
    sol_alloy al{};
    sol_bcs bcs{};
    sol_numerics num{};
    Sizes z{};
    hipStream_t stream = nullptr;
    Mem mem;
    CaseDev cd{};
    double *work[3][NWORK] = {};
    float *work32[3][NWORK32] = {};
    int32_t *csr_cnt = nullptr, *csr_rp[NSYS] = {}, *csr_col[NSYS] = {};
    double *csr_val[NSYS] = {};
    Group *solo = nullptr;
    sol_batch *batch = nullptr;
    bool timing = false;
    bool opt_graph = false;
    int precond = SOL_PRECOND_MG;
    int tprecond = SOL_TPRECOND_AUTO;
    int assembly = SOL_ASSEMBLY_STENCIL;
    int momentum = SOL_MOMENTUM_PLAIN;    // SOL_OPT_MOMENTUM: form of the momentum predictor
    bool mg_fuse = true;                  // SOL_OPT_MG_FUSE: coarse multigrid levels in pairs
    double *mg_pwork = nullptr;           // scratch of the exact-level inverse (set-up)
    double *mg_p64 = nullptr;             // FP64 exact-level inverse (set-up; solves read its FP32 copy)
    // large grids: level mg_nbig (> 0) is solved exactly instead of mg_nglob
    // when the case runs alone; its inverse is built before the first such step
    int mg_nbig = 0;
    bool mg_big_ready = false;
    double *mg_pbig64 = nullptr, *mg_pbigwork = nullptr;
    int64_t redone = 0;                   // steps run a second time (speculative check failed)
    // pressure multigrid hierarchy (FP64 arrays; FP32 copies for mixed precision)
    int mg_nlev = 0, mg_nglob = 0;
    MLevel mg_h[MG_MAXLEV] = {};
    MLevel mg32_h[MG_MAXLEV] = {};
    MLevel *mg_d = nullptr, *mg32_d = nullptr;
    TAcc tacc[SOL_NKCLASS];
    std::vector<TSample> samples;
    std::vector<hipEvent_t> event_pool;
    int64_t last_iters[NSYS] = {};
};

// ------------------------------------------------------------------ groups

// One launch of an iteration: kernel, tiles per stencil width, local memory.
struct Stage {
    int which = 0, cls = 0;
    JTile *tiles_d[2] = {nullptr, nullptr};
    int nt[2] = {0, 0};
    size_t smem[2] = {0, 0};
    bool two[2] = {false, false};        // BiCGSTAB: two Jacobi sweeps (per stencil width)
    bool s1[2] = {false, false};         // BiCGSTAB, one sweep: every solve of the width staged in LDS
};

// A set of solves launched together (one kernel launch serves all of them).
struct JobSet {
    std::vector<KJob> jobs;
    std::vector<int> st_index;          // index into the group's KState array
    std::vector<int> case_of, sys_of;
    KJob *jobs_d = nullptr;
    JTile *tiles_d[2] = {nullptr, nullptr};   // [0] 5-point jobs, [1] 7-point jobs
    int nt[2] = {0, 0};
    hipGraph_t graph = nullptr;          // GCH iterations + advance of the index base
    hipGraphExec_t exec = nullptr;
    int graph_nodes = 0;                 // kernel nodes of the graph
    std::vector<Stage> iter;             // launches of one iteration
    std::vector<Stage> start;            // multigrid: the V-cycle of the start (after its init kernel)
};

struct Phase {
    int kind = K_BICGSTAB;
    bool two[2] = {false, false};        // BiCGSTAB: two Jacobi sweeps, 5- / 7-point systems
    int tcls0 = SOL_KCLASS_BICG_A;       // timing class of the first iteration kernel
    bool mixed = false;
    JobSet main;                         // FP64 solves (plain, or the refinements)
    JobSet inner;                        // mixed precision: FP32 inner solves
    int pred = 1, pred_inner = 1;
    int64_t launched = 0;
    bool pending = false;                // solved speculatively, verdict not read yet
    bool synced = false;                 // the last solve ended with a state copy into slot 0
};

struct Group {
    std::vector<sol_handle *> cs;
    hipStream_t stream = nullptr;
    std::vector<void *> dmem;            // hipMalloc'd chunks of the group arrays
    char *chunk = nullptr;               // the chunk gmalloc currently cuts from
    size_t chunk_size = 0, chunk_used = 0;
    CaseDev *cases_d = nullptr;
    KState *ks_d = nullptr;              // [2 * nks]: solves, then inner solves
    double *red_d = nullptr;
    int32_t *cidx_d = nullptr;           // 0..n-1 (per-case one-workgroup kernels)
    Tile *t_mom[2] = {}, *t_cell[2] = {}, *t_const[2] = {};
    int n_mom[2] = {}, n_cell[2] = {}, n_const[2] = {};
    Phase ph[3];                          // momentum, pressure, solute + energy
    KState *ks_h[2] = {nullptr, nullptr};  // pinned poll buffers
    hipEvent_t ev[2] = {nullptr, nullptr};
    int nks = 0;
    int precision = SOL_PRECISION_FP64;
    sol_handle *timer = nullptr;          // handle that collects kernel timing (solo groups)
    int *kbase_d = nullptr;               // iteration index base of graph-replayed chunks
    bool use_graph = false;
    bool mg_fuse = true;                  // coarse multigrid levels fused in pairs
};

// group arrays come out of 1 MiB chunks (256-byte aligned pieces; a larger
// request gets a chunk of its own), so that building a group takes a few
// hipMalloc calls instead of one per array: a served batch is rebuilt
// whenever its membership changes
constexpr size_t GCHUNK = 1 << 20;
static void *gmalloc(Group &g, size_t bytes)
{
    bytes = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
    if (g.chunk && g.chunk_used + bytes <= g.chunk_size) {
        void *p = g.chunk + g.chunk_used;
        g.chunk_used += bytes;
        return p;
    }
    const size_t sz = std::max(bytes, GCHUNK);
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) return nullptr;
    g.dmem.push_back(p);
    if (sz == GCHUNK || !g.chunk) {
        g.chunk = (char *)p;
        g.chunk_size = sz;
        g.chunk_used = bytes;
    }
    return p;
}

static void group_free(Group *g)
{
    if (!g) return;
    for (auto &P : g->ph)
        for (JobSet *S : {&P.main, &P.inner}) {
            if (S->exec) (void)hipGraphExecDestroy(S->exec);
            if (S->graph) (void)hipGraphDestroy(S->graph);
        }
    for (void *p : g->dmem) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (g->ks_h[i]) (void)hipHostFree(g->ks_h[i]);
        if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
    }
    delete g;
}

template <class T>
static int upload(Group &g, T **dst, const std::vector<T> &src)
{
    *dst = nullptr;
    if (src.empty()) return SOL_OK;
    *dst = (T *)gmalloc(g, sizeof(T) * src.size());
    if (!*dst) return fail(SOL_ENOMEM, "group allocation failed");
    HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return SOL_OK;
}

// partial-sum buffers, tile lists and device copy of a job set
// Tile list of a launch that serves several solves.  The kernels map
// workgroup b (dispatched to XCD b mod 8) to list position
// xcd_tile(b, n): XCD x works through the x-th contiguous eighth of the
// list.  Listing the solves one after another would give a solve that has
// converged (its workgroups exit at once) whole XCDs, and the solves still
// iterating only the others.  Here the x-th eighth of every solve's tiles is
// placed in XCD x's range (tiles of one solve stay contiguous there, so
// neighbour rows stay in that XCD's L2), the remainders dealt round-robin
// so that the range sizes are those xcd_tile expects.
static std::vector<JTile> xcd_order(const std::vector<std::vector<JTile>> &per_solve)
{
    std::vector<std::vector<JTile>> xl(NXCD);
    int next = 0;
    for (const auto &tl : per_solve) {
        const int nt = (int)tl.size(), base = nt / NXCD, extra = nt % NXCD;
        int cnt[NXCD];
        for (int x = 0; x < NXCD; ++x) cnt[x] = base;
        for (int e = 0; e < extra; ++e) cnt[(next + e) % NXCD] += 1;
        next = (next + extra) % NXCD;
        int pos = 0;
        for (int x = 0; x < NXCD; ++x)
            for (int i = 0; i < cnt[x]; ++i) xl[x].push_back(tl[pos++]);
    }
    std::vector<JTile> out;
    for (const auto &l : xl) out.insert(out.end(), l.begin(), l.end());
    return out;
}

// multigrid level solved exactly for case h in group g: a large grid
// stepped alone (its iterations launch bound) uses its larger exact level
// once that inverse is built; in a batch of several cases every case keeps
// the standard one, whose product each case reads in every iteration
static int case_nglob(const Group &g, const sol_handle *h)
{
    return (g.cs.size() == 1 && h->mg_nbig > 0 && h->mg_big_ready) ? h->mg_nbig : h->mg_nglob;
}

// BiCGSTAB preconditioner of a system with nd diagonals: two Jacobi sweeps
// or one.  Automatic: two on 5-point (2D) systems, where halving the
// iterations outweighs the wider gathers; one on 7-point (3D) systems, where
// the 25-cell gathers cost more than the iterations they save.
static bool two_sweeps(int tprecond, int nd)
{
    return tprecond == SOL_TPRECOND_JACOBI2 || (tprecond == SOL_TPRECOND_AUTO && nd == 5);
}

// a two-sweep 5-point FP64 solve goes through LDS when its tile
// neighbourhood fits the LDS budget and its halo (two rows of the grid on
// either side) is at most four times the tile, beyond which staging loads
// more than gathering per row; the choice depends on the case alone, so a
// case gets the same kernels' arithmetic alone and in a batch
static int stage2_fits(bool two5, int rpt, int sx, size_t tsize)
{
    return two5 && 4 * sx + 4 <= 4 * rpt && (size_t)stage2_values(rpt, sx) * tsize <= (size_t)STAGE2_LDS_MAX ? 1 : 0;
}

// a one-sweep 7-point FP64 solve goes through LDS on the same terms, its halo
// (one grid row on either side) at most the tile: at 128x128x64 the A kernel
// of the momentum group measured 46.5 -> 41.3 us per launch, the same
// arithmetic (FP32 inner solves measured slower staged, and stay gathered)
static int stage1_fits(bool one7, int rpt, int sx, size_t tsize)
{
    return one7 && 2 * sx <= rpt && (size_t)stage1_values(rpt, sx) * tsize <= (size_t)STAGE2_LDS_MAX ? 1 : 0;
}

static int finish_set(Group &g, JobSet &S)
{
    size_t total = 0;
    for (auto &J : S.jobs) total += (size_t)J.ntile * 2 * NSLOT;
    double *part = (double *)gmalloc(g, sizeof(double) * std::max<size_t>(total, 1));
    if (!part) return fail(SOL_ENOMEM, "group allocation failed");
    size_t off = 0;
    for (size_t j = 0; j < S.jobs.size(); ++j) {
        S.jobs[j].part = part + off;
        off += (size_t)S.jobs[j].ntile * 2 * NSLOT;
    }
    // Within an XCD's range the workgroups are dispatched in list order, and
    // the two-sweep BiCGSTAB kernels hold two workgroups per CU, fewer than a
    // launch has: the solves that usually iterate longest are listed first,
    // so that the workgroups of a solve that has converged (which exit at
    // once) take the slots left over instead of delaying those of the solves
    // still running.  The solute solve (its matrix is close to diagonal)
    // mostly converges in one iteration while the energy solve takes ten.
    std::vector<std::vector<JTile>> per[2];
    for (int pass = 0; pass < 2; ++pass)
        for (size_t j = 0; j < S.jobs.size(); ++j) {
            if ((S.sys_of[j] == SC) != (pass == 1)) continue;
            const KJob &J = S.jobs[j];
            const int gi = g.cs[S.case_of[j]]->z.nd == 7 ? 1 : 0;
            std::vector<JTile> tl;
            for (int t = 0; t < J.ntile; ++t) tl.push_back({(int)j, t, 0, 0});
            per[gi].push_back(std::move(tl));
        }
    RCHK(upload(g, &S.jobs_d, S.jobs));
    for (int gi = 0; gi < 2; ++gi) {
        const std::vector<JTile> jt = xcd_order(per[gi]);
        RCHK(upload(g, &S.tiles_d[gi], jt));
        S.nt[gi] = (int)jt.size();
    }
    return SOL_OK;
}

// launches of one iteration (and of the multigrid start cycle) of a job set
static int build_stages(Group &g, JobSet &S, int kind, const bool (&two)[2], int fp32)
{
    S.iter.clear();
    S.start.clear();
    auto row_stage = [&](int which, int cls) {
        Stage st;
        st.which = which;
        st.cls = cls;
        for (int gi = 0; gi < 2; ++gi) {
            st.tiles_d[gi] = S.tiles_d[gi];
            st.nt[gi] = S.nt[gi];
            st.two[gi] = two[gi];
        }
        return st;
    };
    if (kind == K_CG) {
        S.iter.push_back(row_stage(KI_CG, SOL_KCLASS_CG));
        return SOL_OK;
    }
    if (kind == K_BICGSTAB) {
        // solves staged in LDS: 5-point two-sweep ones per solve inside the
        // two-sweep kernels; 7-point one-sweep ones through kernels of their
        // own, taken when every 7-point solve of the launch is staged.  The
        // launch of each stencil width reserves the largest tile
        // neighbourhood among its staged solves.
        size_t lds[2] = {0, 0};
        bool all7 = true, any7 = false;
        const size_t ts = fp32 ? sizeof(float) : sizeof(double);
        for (size_t j = 0; j < S.jobs.size(); ++j) {
            const KJob &J = S.jobs[j];
            const bool seven = g.cs[S.case_of[j]]->z.nd == 7;
            if (seven) {
                any7 = true;
                all7 = all7 && J.staged;
            }
            if (!J.staged) continue;
            const size_t v = seven ? (size_t)stage1_values(J.rpt, J.sx) : (size_t)stage2_values(J.rpt, J.sx);
            lds[seven] = std::max(lds[seven], v * ts);
        }
        const bool s1 = any7 && all7 && !two[1];
        S.iter.push_back(row_stage(KI_BICG_B, SOL_KCLASS_BICG_B));
        S.iter.push_back(row_stage(KI_BICG_A, SOL_KCLASS_BICG_A));
        for (Stage &st : S.iter) {
            st.smem[0] = lds[0];
            st.smem[1] = s1 ? lds[1] : 0;
            st.s1[1] = s1;
        }
        return SOL_OK;
    }
    // multigrid CG: pq, down0, down(1..G-1), exact, up(G-1..1), up0; the start
    // cycle is the same without pq, with the start variant of down0.  With
    // fused coarse levels the levels 1..G-1 go in slots of two: a slot at
    // level l runs levels l and l+1 in one launch each way for the solves
    // with l + 1 < G, and level l alone for those with G = l + 1.
    int gmax = 1;
    for (size_t j = 0; j < S.jobs.size(); ++j) gmax = std::max(gmax, case_nglob(g, g.cs[S.case_of[j]]));
    const bool fuse = g.mg_fuse;
    std::vector<Stage> down, up;          // in the down order; up runs them reversed
    for (int l = 1; l < gmax; l += fuse ? 2 : 1) {
        std::vector<std::vector<JTile>> per[2][2];   // [single, pair][stencil width]
        for (size_t j = 0; j < S.jobs.size(); ++j) {
            const sol_handle *h = g.cs[S.case_of[j]];
            const int G = case_nglob(g, h);
            if (G <= l) continue;
            const int gi = h->z.nd == 7 ? 1 : 0;
            const int pair = fuse && G >= l + 2 ? 1 : 0;
            const int nt = pair ? mg_fused_bricks(h->z.dim, h->mg_h[l + 1]) : h->mg_h[l].ntile;
            std::vector<JTile> tl;
            for (int t = 0; t < nt; ++t) tl.push_back({(int)j, t, l, 0});
            per[pair][gi].push_back(std::move(tl));
        }
        for (int pair = 1; pair >= 0; --pair) {
            Stage st;
            st.which = pair ? KI_MG_DOWN2 : KI_MG_DOWN;
            st.cls = SOL_KCLASS_MG_COARSE;
            for (int gi = 0; gi < 2; ++gi) {
                const std::vector<JTile> jt = xcd_order(per[pair][gi]);
                if (!jt.empty()) RCHK(upload(g, &st.tiles_d[gi], jt));
                st.nt[gi] = (int)jt.size();
            }
            if (st.nt[0] + st.nt[1] == 0) continue;
            down.push_back(st);
            st.which = pair ? KI_MG_UP2 : KI_MG_UP;
            up.push_back(st);
        }
    }
    Stage exact;
    exact.which = KI_MG_EXACT;
    exact.cls = SOL_KCLASS_MG_COARSE;
    {
        std::vector<JTile> jt[2];
        for (size_t j = 0; j < S.jobs.size(); ++j) {
            const sol_handle *h = g.cs[S.case_of[j]];
            const int gi = h->z.nd == 7 ? 1 : 0;
            const int L = case_nglob(g, h);
            for (int t = 0; t < ceil_div(h->mg_h[L].n, MG_XROWS); ++t) jt[gi].push_back({(int)j, t, L, 0});
        }
        for (int gi = 0; gi < 2; ++gi) {
            RCHK(upload(g, &exact.tiles_d[gi], jt[gi]));
            exact.nt[gi] = (int)jt[gi].size();
        }
    }
    auto cycle = [&](std::vector<Stage> &out, int down0) {
        out.push_back(row_stage(down0, SOL_KCLASS_MG_DOWN0));
        for (const Stage &st : down) out.push_back(st);
        out.push_back(exact);
        for (size_t i = up.size(); i-- > 0;) out.push_back(up[i]);
        out.push_back(row_stage(KI_MG_UP0, SOL_KCLASS_MG_UP0));
    };
    S.iter.push_back(row_stage(KI_MG_PQ, SOL_KCLASS_MG_PQ));
    cycle(S.iter, KI_MG_DOWN0);
    cycle(S.start, KI_MG_DOWN0_INIT);
    return SOL_OK;
}

// level tables of the pressure multigrid with the current tiles of the
// level-0 kernels (tile size is process-wide per size class)
static int mg_upload(sol_handle *h)
{
    const int cpt0 = mg_cells_per_tile(h->z.nsys[SP], h->z.nd, h->mg_h[0].cn);
    for (MLevel *t : {h->mg_h, h->mg32_h}) {
        t[0].cpt = cpt0;
        t[0].ntile = t[0].cn ? ceil_div(t[0].cn, cpt0) : 0;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(h->mg_d, h->mg_h, sizeof(MLevel) * MG_MAXLEV, hipMemcpyHostToDevice));
    if (h->mg32_d) HIPCHK(hipMemcpy(h->mg32_d, h->mg32_h, sizeof(MLevel) * MG_MAXLEV, hipMemcpyHostToDevice));
    return SOL_OK;
}

// inner relative tolerance of the FP32 solves of the refinement
static double inner_tol(double tol) { return std::max(tol, 1e-5); }

static int group_build(Group &g)
{
    const int n = (int)g.cs.size();
    g.nks = n * NSYS;
    g.precision = g.cs[0]->num.precision;
    const bool mixed = g.precision == SOL_PRECISION_MIXED;
    g.ks_d = (KState *)gmalloc(g, sizeof(KState) * 2 * g.nks);
    g.red_d = (double *)gmalloc(g, sizeof(double) * 16 * n);
    g.kbase_d = (int *)gmalloc(g, 256);
    if (!g.ks_d || !g.red_d || !g.kbase_d) return fail(SOL_ENOMEM, "group allocation failed");
    HIPCHK(hipMemset(g.kbase_d, 0, 256));
    HIPCHK(hipMemset(g.red_d, 0, sizeof(double) * 16 * n));
    std::vector<CaseDev> cdv(n);
    std::vector<KState> ksv(2 * g.nks);
    for (auto &k : ksv) { std::memset(&k, 0, sizeof(k)); k.status = K_IDLE; }
    std::vector<Tile> mom[2], cell[2], cst[2];
    const bool mg = g.cs[0]->precond == SOL_PRECOND_MG;
    for (int c = 0; c < n; ++c) RCHK(mg_upload(g.cs[c]));
    for (int c = 0; c < n; ++c) {
        sol_handle *h = g.cs[c];
        CaseDev d = h->cd;
        d.ks = g.ks_d + c * NSYS;
        d.red = g.red_d + 16 * c;
        cdv[c] = d;
        const int gi = h->z.dim == 3 ? 1 : 0;
        for (int s = 0; s < h->z.dim; ++s)
            for (int t = 0; t < ceil_div(h->z.nsys[s], TILE); ++t) mom[gi].push_back({c, s, t, 0});
        for (int t = 0; t < h->z.ntile_cell; ++t) cell[gi].push_back({c, SC, t, 0});
        const int cs_list[5] = {SU, SV, SW, SP, ST};
        for (int s : cs_list)
            for (int t = 0; t < ceil_div(h->z.nsys[s], TILE); ++t) cst[gi].push_back({c, s, t, 0});
        for (int s = 0; s < NSYS; ++s) {
            const double tol = s == SP ? h->num.tol_p : h->num.tol_t;
            KState &k = ksv[c * NSYS + s];
            k.tol2 = tol * tol;
            k.max_iter = h->num.max_iter;
            KState &ki = ksv[g.nks + c * NSYS + s];
            ki.tol2 = inner_tol(tol) * inner_tol(tol);
            // FP32 Krylov can stagnate near its rounding floor: bound one inner
            // solve well above the CG count the grid needs (~ a few n per axis)
            ki.max_iter = std::min(h->num.max_iter, 20 * (h->z.nx + h->z.ny + h->z.nz) + 100);
        }
    }
    RCHK(upload(g, &g.cases_d, cdv));
    {
        std::vector<int32_t> ci(n);
        for (int c = 0; c < n; ++c) ci[c] = c;
        RCHK(upload(g, &g.cidx_d, ci));
    }
    HIPCHK(hipMemcpy(g.ks_d, ksv.data(), sizeof(KState) * 2 * g.nks, hipMemcpyHostToDevice));
    for (int gi = 0; gi < 2; ++gi) {
        RCHK(upload(g, &g.t_mom[gi], mom[gi]));
        RCHK(upload(g, &g.t_cell[gi], cell[gi]));
        RCHK(upload(g, &g.t_const[gi], cst[gi]));
        g.n_mom[gi] = (int)mom[gi].size();
        g.n_cell[gi] = (int)cell[gi].size();
        g.n_const[gi] = (int)cst[gi].size();
    }
    // solve phases
    const int phase_sys[3][3] = {{SU, SV, SW}, {SP, -1, -1}, {SC, ST, -1}};
    for (int p = 0; p < 3; ++p) {
        Phase &P = g.ph[p];
        P.kind = p == 1 ? (mg ? K_MGCG : K_CG) : K_BICGSTAB;
        for (int gi = 0; gi < 2; ++gi) P.two[gi] = P.kind == K_BICGSTAB && two_sweeps(g.cs[0]->tprecond, gi ? 7 : 5);
        P.tcls0 = p == 1 ? (mg ? SOL_KCLASS_MG_PQ : SOL_KCLASS_CG) : SOL_KCLASS_BICG_A;
        P.mixed = mixed;
        for (int c = 0; c < n; ++c) {
            sol_handle *h = g.cs[c];
            for (int k = 0; k < 3; ++k) {
                const int s = phase_sys[p][k];
                if (s < 0 || h->z.nsys[s] == 0) continue;
                KJob J;
                std::memset(&J, 0, sizeof(J));
                J.n = h->z.nsys[s];
                J.sx = h->z.sdim[s][0];
                J.sxy = h->z.sdim[s][0] * h->z.sdim[s][1];
                J.rpt = rows_per_tile(J.n, h->z.nd);
                J.ntile = ceil_div(J.n, J.rpt);
                J.kind = P.kind;
                if (P.kind == K_MGCG) {
                    J.nlev = h->mg_nlev;
                    J.nglob = case_nglob(g, h);
                    J.lev = h->mg_d;
                    J.ntile = h->mg_h[0].ntile;
                    J.rpt = ceil_div(J.n, J.ntile);
                }
                J.A = h->cd.A[s];
                J.b = h->cd.b[s];
                J.minv = h->cd.minv[s];
                const int ws = p == 0 ? s : (p == 1 ? 0 : (s == SC ? 0 : 1));
                // u*, phi and T*: the initial guess is written into the
                // solution buffer itself (k_guess_mom before the momentum
                // solves, k_guess before the pressure solve)
                if (p == 0) { J.x = h->cd.us[s]; J.x0 = h->cd.us[s]; }
                else if (p == 1) { J.x = h->cd.phi; J.x0 = h->cd.phi; }
                else if (s == SC) { J.x = h->cd.Cnew; J.x0 = h->cd.C; }
                else { J.x = h->cd.Tstar; J.x0 = h->cd.Tstar; }
                J.st = g.ks_d + c * NSYS + s;
                if (!mixed) {
                    J.role = ROLE_PLAIN;
                    J.r = h->work[ws][0]; J.rh = h->work[ws][1];
                    J.p0 = h->work[ws][2]; J.p1 = h->work[ws][3];
                    J.v0 = h->work[ws][4]; J.v1 = h->work[ws][5];
                    J.t = h->work[ws][6]; J.r1 = h->work[ws][7];
                } else {
                    // refinement: FP64 residual sweeps; aux = FP32 residual, t = FP32 correction
                    KState *ist = g.ks_d + g.nks + c * NSYS + s;
                    J.role = ROLE_REFINE;
                    J.aux = h->work32[ws][8];
                    J.t = h->work32[ws][7];
                    J.partner = ist;
                    KJob I = J;
                    I.role = ROLE_INNER;
                    I.A = h->cd.A32[s];
                    I.minv = h->cd.minv32[s];
                    I.b = h->work32[ws][8];
                    I.x = h->work32[ws][7];
                    I.x0 = nullptr;
                    I.aux = nullptr;
                    I.r = h->work32[ws][0]; I.rh = h->work32[ws][1];
                    I.p0 = h->work32[ws][2]; I.p1 = h->work32[ws][3];
                    I.v0 = h->work32[ws][4]; I.v1 = h->work32[ws][5];
                    I.t = h->work32[ws][6]; I.r1 = h->work32[ws][9];
                    I.st = ist;
                    I.partner = J.st;
                    I.lev = h->mg32_d;
                    I.staged = 0;     // FP32: gathering per row measured faster
                    P.inner.jobs.push_back(I);
                    P.inner.st_index.push_back(g.nks + c * NSYS + s);
                    P.inner.case_of.push_back(c);
                    P.inner.sys_of.push_back(s);
                }
                J.staged = h->z.nd == 5 ? stage2_fits(P.two[0], J.rpt, J.sx, sizeof(double))
                                        : stage1_fits(P.kind == K_BICGSTAB && !P.two[1], J.rpt, J.sx, sizeof(double));
                P.main.jobs.push_back(J);
                P.main.st_index.push_back(c * NSYS + s);
                P.main.case_of.push_back(c);
                P.main.sys_of.push_back(s);
            }
        }
        RCHK(finish_set(g, P.main));
        RCHK(build_stages(g, P.main, P.kind, P.two, 0));
        if (mixed) {
            RCHK(finish_set(g, P.inner));
            RCHK(build_stages(g, P.inner, P.kind, P.two, 1));
        }
        P.pred = P.pred_inner = p == 1 ? (mg ? 24 : 64) : 2;
    }
    for (int i = 0; i < 2; ++i) {
        HIPCHK(hipHostMalloc((void **)&g.ks_h[i], sizeof(KState) * 2 * g.nks, hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&g.ev[i], hipEventDisableTiming));
    }
    return SOL_OK;
}

static int group_create(const std::vector<sol_handle *> &cs, Group **out)
{
    Group *g = new Group();
    g->cs = cs;
    g->stream = cs[0]->stream;
    g->mg_fuse = cs[0]->mg_fuse;          // a batch follows its first handle
    int rc = group_build(*g);
    if (rc != SOL_OK) { group_free(g); return rc; }
    *out = g;
    return SOL_OK;
}

// ------------------------------------------------------------ timing helpers

static hipEvent_t take_event(sol_handle *h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Turn the pending samples into durations (after a synchronising poll whose
// states are ks).  Every launch counts; the bytes of a Krylov launch are
// those of the solves still iterating at it (iteration index below the
// solve's final count), so a launch queued after convergence, which exits at
// once, adds its time and no bytes, as a profiler would see it.  Samples
// of solves that restarted are dropped (their iteration indices are shifted).
static void collect_samples(Group &g, const KState *ks)
{
    sol_handle *h = g.timer;
    if (!h) return;
    for (auto &s : h->samples) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s.a, s.b) != hipSuccess) continue;
        double bytes = 0.0;
        bool valid = true;
        if (s.set) {
            double rows = 0.0, rows_half = 0.0, rows_nom = 0.0;
            int nd = 5, dim = 2;
            for (size_t j = 0; j < s.set->jobs.size(); ++j) {
                const KState &k = ks[s.set->st_index[j]];
                if (k.restarts != 0) valid = false;
                if (s.iter < k.it) {
                    nd = g.cs[s.set->case_of[j]]->z.nd;
                    dim = g.cs[s.set->case_of[j]]->z.dim;
                    // the last A launch of a solve that stopped at its half step
                    if (s.cls == SOL_KCLASS_BICG_A && k.half && s.iter == k.it - 1) rows_half += s.set->jobs[j].n;
                    else if (b_without_m(s, s.set->jobs[j], nd)) rows_nom += s.set->jobs[j].n;
                    else rows += s.set->jobs[j].n;
                }
            }
            bytes = (rows * row_bytes(s.cls, nd, dim, s.tsize) + rows_half * half_exit_bytes(nd, s.two, s.tsize) +
                     rows_nom * (row_bytes(s.cls, nd, dim, s.tsize) - s.tsize)) *
                    s.count;
        } else {
            for (auto *c : g.cs) {
                const double rows = s.cls == SOL_KCLASS_ASM_MOM
                                        ? (double)(c->z.nsys[0] + c->z.nsys[1] + c->z.nsys[2])
                                        : (double)c->z.ncell;
                bytes += rows * row_bytes(s.cls, c->z.nd, c->z.dim, 8, s.fwd);
            }
        }
        if (valid) {
            h->tacc[s.cls].n += s.count;
            h->tacc[s.cls].ms += ms;
            h->tacc[s.cls].bytes += bytes;
        }
        h->event_pool.push_back(s.a);
        h->event_pool.push_back(s.b);
    }
    h->samples.clear();
}

// ------------------------------------------------------------------ solves

// Graph replay of iteration chunks: a graph holds GCH iterations of a job set
// (kernel nodes reading the iteration index from the device base plus a
// fixed offset) followed by a node that advances the base by GCH.  Built
// node by node (no stream capture: the library may run on the legacy
// default stream) on first use and replayed for every chunk.
constexpr int GCH = 16;

static int build_chunk_graph(Group &g, Phase &P, JobSet &S, int fp32)
{
    (void)P;
    HIPCHK(hipGraphCreate(&S.graph, 0));
    hipGraphNode_t prev = nullptr;
    for (int i = 0; i < GCH; ++i)
        for (const Stage &st : S.iter)
            for (int gi = 0; gi < 2; ++gi) {
                if (st.nt[gi] <= 0) continue;
                const KJob *jobs = S.jobs_d;
                const JTile *tiles = st.tiles_d[gi];
                const int *kb = g.kbase_d;
                int koff = i;
                void *args[] = {(void *)&jobs, (void *)&tiles, (void *)&kb, (void *)&koff};
                hipKernelNodeParams kp;
                std::memset(&kp, 0, sizeof(kp));
                kp.func = (void *)kiter_fn(st.which, gi ? 7 : 5, fp32, st.two[gi], st.s1[gi]);
                kp.gridDim = dim3((unsigned)st.nt[gi]);
                kp.blockDim = dim3(TILE);
                kp.sharedMemBytes = (unsigned)st.smem[gi];
                kp.kernelParams = args;
                kp.extra = nullptr;
                hipGraphNode_t node;
                HIPCHK(hipGraphAddKernelNode(&node, S.graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
                prev = node;
                ++S.graph_nodes;
            }
    {
        int *kb = g.kbase_d;
        int m = GCH;
        void *args[] = {(void *)&kb, (void *)&m};
        hipKernelNodeParams kp;
        std::memset(&kp, 0, sizeof(kp));
        kp.func = (void *)kbase_add_fn();
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(64);
        kp.kernelParams = args;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, S.graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        ++S.graph_nodes;
    }
    HIPCHK(hipGraphInstantiate(&S.exec, S.graph, nullptr, nullptr, 0));
    return SOL_OK;
}

// one launch per stencil width of a stage at iteration index koff (kb NULL);
// with events ta / tb (a stage of one stencil width only) the dispatch
// itself is time-stamped, as a profiler sees it
static int launch_stage(Group &g, const JobSet &S, const Stage &st, int fp32, int koff, hipEvent_t ta = nullptr,
                        hipEvent_t tb = nullptr)
{
    for (int gi = 0; gi < 2; ++gi) {
        if (st.nt[gi] <= 0) continue;
        const KJob *jobs = S.jobs_d;
        const JTile *tiles = st.tiles_d[gi];
        const int *kb = nullptr;
        void *args[] = {(void *)&jobs, (void *)&tiles, (void *)&kb, (void *)&koff};
        const void *fn = kiter_fn(st.which, gi ? 7 : 5, fp32, st.two[gi], st.s1[gi]);
        note_dispatch(1);
        if (ta && tb)
            HIPCHK(hipExtLaunchKernel(fn, dim3((unsigned)st.nt[gi]), dim3(TILE), args, st.smem[gi], g.stream, ta, tb, 0));
        else
            HIPCHK(hipLaunchKernel(fn, dim3((unsigned)st.nt[gi]), dim3(TILE), args, st.smem[gi], g.stream));
    }
    return SOL_OK;
}

// (re)start the solves of S at iteration index k (mode 0: all, mode 1: those
// in K_RESTART); multigrid: init kernel, then the start V-cycle at k - 1
static int start_solves(Group &g, Phase &P, JobSet &S, int fp32, int k, int mode)
{
    if (P.kind != K_MGCG) {
        for (int gi = 0; gi < 2; ++gi)
            launch_kinit(P.kind, gi ? 7 : 5, fp32, P.two[gi], !S.iter.empty() && S.iter[0].s1[gi], S.jobs_d,
                         S.tiles_d[gi], S.nt[gi], k, mode, S.iter.empty() ? 0 : S.iter[0].smem[gi], g.stream);
        return SOL_OK;
    }
    for (int gi = 0; gi < 2; ++gi) launch_mg_init(gi ? 7 : 5, fp32, S.jobs_d, S.tiles_d[gi], S.nt[gi], k, mode, g.stream);
    for (const Stage &st : S.start) RCHK(launch_stage(g, S, st, fp32, k - 1));
    return SOL_OK;
}

// Timing: CG iterations are timed in windows of TWIN consecutive launches
// (one event pair per window; per-launch events would add their own
// latency), BiCGSTAB and multigrid kernels one launch at a time with the
// events stamped by the dispatch itself (hipExtLaunchKernel), every launch
// (so the average covers the same launches as a profiler's).
constexpr int TWIN = 16;

static int enqueue_iters(Group &g, Phase &P, JobSet &S, int fp32, int nits, int &k)
{
    sol_handle *tm = g.timer;
    if (g.use_graph && !tm && nits >= GCH) {
        if (!S.exec) RCHK(build_chunk_graph(g, P, S, fp32));
        launch_kbase_set(g.kbase_d, k, g.stream);
        const int chunks = ceil_div(nits, GCH);
        for (int c = 0; c < chunks; ++c) HIPCHK(hipGraphLaunch(S.exec, g.stream));
        note_dispatch((long)chunks * S.graph_nodes);
        k += chunks * GCH;
        P.launched += chunks * GCH;
        return SOL_OK;
    }
    hipEvent_t wa = nullptr, wb = nullptr;
    int wend = -1;
    for (int it = 0; it < nits; ++it) {
        if (tm && P.kind == K_CG && wend < 0 && k % (2 * TWIN) == 0 && nits - it >= TWIN) {
            wa = take_event(tm);
            wb = take_event(tm);
            if (wa && wb) {
                (void)hipEventRecord(wa, g.stream);
                wend = k + TWIN - 1;
            }
        }
        const bool sample = tm && P.kind != K_CG;
        for (const Stage &st : S.iter) {
            hipEvent_t a = nullptr, b = nullptr;
            if (sample && (st.nt[0] <= 0 || st.nt[1] <= 0)) { a = take_event(tm); b = take_event(tm); }
            RCHK(launch_stage(g, S, st, fp32, k, a, b));
            if (a && b) {
                const int w = st.nt[0] > 0 ? 0 : 1;
                tm->samples.push_back({st.cls, (int64_t)k, &S, fp32 ? 4 : 8, a, b, 1, st.two[w], st.s1[w]});
            }
        }
        if (k == wend) {
            (void)hipEventRecord(wb, g.stream);
            tm->samples.push_back({P.tcls0, (int64_t)k, &S, fp32 ? 4 : 8, wa, wb, TWIN});
            wend = -1;
        }
        k += 1;
        P.launched += 1;
    }
    return SOL_OK;
}

static int poll_enqueue(Group &g, int slot)
{
    note_dispatch(1);
    HIPCHK(hipMemcpyAsync(g.ks_h[slot], g.ks_d, sizeof(KState) * 2 * g.nks, hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipEventRecord(g.ev[slot], g.stream));
    return SOL_OK;
}

static int poll_wait(Group &g, int slot)
{
    HIPCHK(hipEventSynchronize(g.ev[slot]));
    return SOL_OK;
}

static bool any_status(const Group &g, const JobSet &S, int slot, int status)
{
    for (int idx : S.st_index)
        if (g.ks_h[slot][idx].status == status) return true;
    return false;
}

// does any solve of S still iterate?  gate (inner solves): only those whose
// refinement was RUNNING at the last synchronising poll (slot gslot)
static bool any_running(const Group &g, const JobSet &S, int slot, const JobSet *gate, int gslot)
{
    for (size_t j = 0; j < S.st_index.size(); ++j) {
        if (gate && g.ks_h[gslot][gate->st_index[j]].status != K_RUNNING) continue;
        if (g.ks_h[slot][S.st_index[j]].status == K_RUNNING) return true;
    }
    return false;
}

// Queue iteration chunks of the solves in S until none is RUNNING.  While
// the host inspects chunk i the device runs chunk i+1.  Returns the slot
// holding the newest states; with wait_last false it returns as soon as the
// states of chunk i show no solve RUNNING, chunk i+1 (no-ops by then) and
// its state copy still queued, and the slot is that of chunk i.
static int iterate(Group &g, Phase &P, JobSet &S, int fp32, int pred, int &k, const JobSet *gate,
                   int gslot, int *out_slot, bool wait_last = true)
{
    int slot = gslot ^ 1;
    const int first = std::max(1, pred - pred / 8);
    const int later = std::max(1, pred / 16);
    RCHK(enqueue_iters(g, P, S, fp32, first, k));
    RCHK(poll_enqueue(g, slot));
    for (;;) {
        RCHK(enqueue_iters(g, P, S, fp32, later, k));
        RCHK(poll_enqueue(g, slot ^ 1));
        RCHK(poll_wait(g, slot));
        if (!any_running(g, S, slot, gate, gslot)) {
            if (!wait_last) {
                *out_slot = slot;
                return SOL_OK;
            }
            RCHK(poll_wait(g, slot ^ 1));
            *out_slot = slot ^ 1;
            return SOL_OK;
        }
        slot ^= 1;
    }
}

static void record_iters(Group &g, const JobSet &S, int slot, int *mx)
{
    for (size_t j = 0; j < S.jobs.size(); ++j) {
        const KState &ks = g.ks_h[slot][S.st_index[j]];
        *mx = std::max(*mx, (int)ks.it);
        g.cs[S.case_of[j]]->last_iters[S.sys_of[j]] = ks.it;
    }
}

// plain FP64 solves.  speculate: once every solve has converged by its
// recurrence, the check of the true residual (k_kfinish, or k_mg_finish for
// the multigrid solves, then k_kdecide) is queued and the call returns
// without waiting for its verdict; the caller reads the verdict (K_DONE, or
// K_RESTART) from a later state copy before anything is committed.
static bool all_converged(const Group &g, const JobSet &S, int slot)
{
    for (int idx : S.st_index) {
        const int st = g.ks_h[slot][idx].status;
        if (st != K_CONVERGED && st != K_ZERO) return false;
    }
    return true;
}

static int solve_plain(Group &g, Phase &P, bool speculate)
{
    JobSet &S = P.main;
    int k = 0;                       // host iteration index of the next launch
    P.launched = 0;
    P.pending = false;
    RCHK(start_solves(g, P, S, 0, k, 0));
    int rc = SOL_OK;
    for (int round = 0; round < 64; ++round) {
        int slot;
        const bool fast = speculate && round == 0;
        // the state copy after k_kdecide below follows the chunk queued
        // ahead on the stream, so the host need not wait for that chunk
        RCHK(iterate(g, P, S, 0, round == 0 ? P.pred : std::max(2, P.pred / 8), k, nullptr, 1, &slot, false));
        for (int gi = 0; gi < 2; ++gi) {
            if (P.kind == K_MGCG) launch_mg_finish(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], g.stream);
            else launch_kfinish(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], g.stream);
        }
        launch_kdecide(S.jobs_d, (int)S.jobs.size(), g.stream);
        if (fast && all_converged(g, S, slot)) {
            int mx = 1;
            record_iters(g, S, slot, &mx);
            P.pred = mx;
            P.pending = true;
            HIPCHK(hipGetLastError());
            return SOL_OK;
        }
        RCHK(poll_enqueue(g, 0));
        RCHK(poll_wait(g, 0));
        HIPCHK(hipGetLastError());
        if (any_status(g, S, 0, K_NONFINITE)) { rc = fail(SOL_ENONFINITE, "non-finite value in a linear solve"); break; }
        if (any_status(g, S, 0, K_FAILED)) {
            for (size_t j = 0; j < S.jobs.size(); ++j) {
                const KState &ks = g.ks_h[0][S.st_index[j]];
                if (ks.status == K_FAILED) {
                    rc = fail(SOL_ENOCONV, "linear solve did not converge (case %d, system %d, %d iterations, "
                                           "%d restarts, ||r||/||b|| = %.3e by the recurrence, %.3e true)",
                              S.case_of[j], S.sys_of[j], ks.it, ks.restarts,
                              ks.bb > 0 ? std::sqrt(ks.rr / ks.bb) : 0.0, ks.bb > 0 ? std::sqrt(ks.tr2 / ks.bb) : 0.0);
                    break;
                }
            }
            break;
        }
        if (!any_status(g, S, 0, K_RESTART)) break;
        RCHK(start_solves(g, P, S, 0, k, 1));
        if (round == 63) rc = fail(SOL_ENOCONV, "linear solve kept restarting");
    }
    int mx = 1;
    record_iters(g, S, 0, &mx);
    P.pred = mx;
    if (g.timer) collect_samples(g, g.ks_h[0]);
    return rc;
}

// mixed precision: FP64 residual sweeps around FP32 inner solves
static int solve_mixed(Group &g, Phase &P)
{
    JobSet &S = P.main, &I = P.inner;
    const int nj = (int)S.jobs.size();
    const int max_outer = 60;
    P.launched = 0;
    for (int gi = 0; gi < 2; ++gi) {
        if (P.kind == K_MGCG) launch_mg_ir_resid(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], 0, g.stream);
        else launch_ir_resid(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], 0, g.stream);
    }
    launch_ir_decide(S.jobs_d, nj, 0, max_outer, g.stream);
    RCHK(poll_enqueue(g, 0));
    // Each sweep's inner solves are started right behind the verdict copy,
    // before the host has read it: the start kernels of a solve whose
    // refinement is no longer RUNNING return at once (outer_idle), so the
    // device runs the starts while the host waits for the verdict.
    int k = 0;
    RCHK(start_solves(g, P, I, 1, k, 0));
    RCHK(poll_wait(g, 0));
    int mx_inner = 1;
    for (int outer = 0; outer < max_outer + 1; ++outer) {
        if (!any_status(g, S, 0, K_RUNNING)) break;
        // the chunk queued after the one that showed no inner solve running
        // is left to run (its launches return at once) while the host queues
        // the refinement kernels behind it
        int slot;
        RCHK(iterate(g, P, I, 1, P.pred_inner, k, &S, 0, &slot, false));
        // an inner solve that broke down (K_RESTART) continues from its x
        // with a fresh residual before its correction is applied
        for (int rs = 0; rs < 8 && any_status(g, I, slot, K_RESTART); ++rs) {
            RCHK(start_solves(g, P, I, 1, k, 1));
            RCHK(iterate(g, P, I, 1, std::max(2, P.pred_inner / 4), k, &S, 0, &slot, false));
        }
        for (int gi = 0; gi < 2; ++gi) launch_ir_update(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], g.stream);
        for (int gi = 0; gi < 2; ++gi) {
            if (P.kind == K_MGCG) launch_mg_ir_resid(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], 1, g.stream);
            else launch_ir_resid(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], 1, g.stream);
        }
        launch_ir_decide(S.jobs_d, nj, 1, max_outer, g.stream);
        RCHK(poll_enqueue(g, 0));
        k = 0;
        RCHK(start_solves(g, P, I, 1, k, 0));
        RCHK(poll_wait(g, 0));
        HIPCHK(hipGetLastError());
        for (size_t j = 0; j < I.jobs.size(); ++j) mx_inner = std::max(mx_inner, (int)g.ks_h[0][I.st_index[j]].it);
        if (g.timer) collect_samples(g, g.ks_h[0]);
    }
    for (int gi = 0; gi < 2; ++gi) launch_ir_update(gi ? 7 : 5, S.jobs_d, S.tiles_d[gi], S.nt[gi], g.stream);
    launch_ir_close(S.jobs_d, nj, g.stream);
    RCHK(poll_enqueue(g, 0));
    RCHK(poll_wait(g, 0));
    HIPCHK(hipGetLastError());
    P.pred_inner = mx_inner;
    int mx = 1;
    record_iters(g, S, 0, &mx);
    P.pred = mx;
    if (any_status(g, S, 0, K_NONFINITE)) return fail(SOL_ENONFINITE, "non-finite value in a linear solve");
    for (size_t j = 0; j < S.jobs.size(); ++j) {
        const KState &ks = g.ks_h[0][S.st_index[j]];
        if (ks.status == K_FAILED || ks.status == K_RUNNING) {
            const KState &ki = g.ks_h[0][I.st_index[j]];
            return fail(SOL_ENOCONV,
                        "refinement did not reach the tolerance (case %d, system %d, %d sweeps, %d inner "
                        "iterations, ||r||/||b|| = %.3e, last inner solve: status %d after %d iterations)",
                        S.case_of[j], S.sys_of[j], ks.outer, ks.inner_total,
                        ks.bb > 0 ? std::sqrt(ks.rr / ks.bb) : 0.0, ki.status, ki.it);
        }
    }
    if (g.timer) collect_samples(g, g.ks_h[0]);
    return SOL_OK;
}

static int group_solve(Group &g, Phase &P, bool speculate = false)
{
    P.pending = false;
    P.synced = false;
    if (P.main.jobs.empty()) return SOL_OK;
    const int rc = P.mixed ? solve_mixed(g, P) : solve_plain(g, P, speculate);
    // every other way out of a solve ends with a state copy into slot 0
    P.synced = rc == SOL_OK && !P.pending;
    return rc;
}

// verdict of a phase solved speculatively, from the newest state copy
// (slot 0): SOL_OK when every solve passed its true-residual check
constexpr int STEP_REDO = 1000;     // internal: redo the step without speculation
static int phase_verdict(const Group &g, const Phase &P)
{
    if (!P.pending) return SOL_OK;
    for (int idx : P.main.st_index)
        if (g.ks_h[0][idx].status != K_DONE) return STEP_REDO;
    return SOL_OK;
}

template <class F>
static void timed(Group &g, int cls, F launch, bool fwd = false)
{
    sol_handle *tm = g.timer;
    hipEvent_t a = nullptr, b = nullptr;
    if (tm) { a = take_event(tm); b = take_event(tm); }
    if (a && b) (void)hipEventRecord(a, g.stream);
    launch();
    if (a && b) {
        (void)hipEventRecord(b, g.stream);
        tm->samples.push_back({cls, 0, nullptr, 8, a, b, 1, false, false, fwd});
    }
}

// one time step (Algorithm 1) for every case of the group
// One step.  With speculate, the momentum and pressure solves hand over to
// the next stage without waiting for their true-residual verdict (the host
// would otherwise wait for the device to drain twice per solve); the
// verdicts arrive with the state copy that ends the transport solves and
// are checked before the commit kernel is queued.  Nothing the step has
// written before the commit is a field of level n, so a step whose verdict
// asks for a restart is simply run again without speculation.
static int group_step_once(Group &g, bool speculate)
{
    hipStream_t s = g.stream;
    // 1: momentum predictor
    const int fwd = g.cs[0]->assembly == SOL_ASSEMBLY_FORWARD;
    timed(g, SOL_KCLASS_ASM_MOM, [&] {
        for (int gi = 0; gi < 2; ++gi) launch_asm_momentum(gi ? 3 : 2, g.cases_d, g.t_mom[gi], g.n_mom[gi], s, fwd);
    }, fwd != 0);
    for (int gi = 0; gi < 2; ++gi) launch_guess_mom(g.cases_d, g.t_mom[gi], g.n_mom[gi], s);
    RCHK(group_solve(g, g.ph[0], speculate));
    // 2: pressure correction (and the initial guesses of phi and T*; the
    // guess kernel removes the rhs mean)
    for (int gi = 0; gi < 2; ++gi) launch_div_rhs(gi ? 3 : 2, g.cases_d, g.t_cell[gi], g.n_cell[gi], 1, s);
    launch_case_mean(g.cases_d, g.cidx_d, (int)g.cs.size(), s);
    for (int gi = 0; gi < 2; ++gi) launch_guess(g.cases_d, g.t_cell[gi], g.n_cell[gi], s);
    RCHK(group_solve(g, g.ph[1], speculate));
    // 3: projection
    for (int gi = 0; gi < 2; ++gi) launch_project(g.cases_d, g.t_mom[gi], g.n_mom[gi], s);
    // 4-6: solute and energy systems (both only need u^{n+1})
    timed(g, SOL_KCLASS_ASM_TRN, [&] {
        for (int gi = 0; gi < 2; ++gi)
            launch_asm_transport(gi ? 3 : 2, g.cases_d, g.t_cell[gi], g.n_cell[gi], 1, s, fwd);
    }, fwd != 0);
    RCHK(group_solve(g, g.ph[2]));
    if (g.ph[0].pending || g.ph[1].pending) {
        if (!g.ph[2].synced) {
            RCHK(poll_enqueue(g, 0));
            RCHK(poll_wait(g, 0));
        }
        RCHK(phase_verdict(g, g.ph[0]));
        RCHK(phase_verdict(g, g.ph[1]));
    }
    // 7-8: phase update, C_l, C_s; commit level n+1
    timed(g, SOL_KCLASS_PHASE, [&] {
        for (int gi = 0; gi < 2; ++gi) launch_phase_commit(gi ? 3 : 2, g.cases_d, g.t_cell[gi], g.n_cell[gi], s);
    });
    launch_case_stats(g.cases_d, g.cidx_d, (int)g.cs.size(), s);
    HIPCHK(hipGetLastError());
    return SOL_OK;
}

static int group_step(Group &g)
{
    // speculation needs the plain FP64 solves; timing runs take every
    // verdict in order
    const bool speculate = !g.timer && !g.ph[0].mixed && !g.ph[1].mixed;
    const int rc = group_step_once(g, speculate);
    if (rc != STEP_REDO) return rc;
    // the step buffers and the solution history hold a discarded attempt
    for (sol_handle *h : g.cs) ++h->redone;
    launch_hist_reset(g.cases_d, (int)g.cs.size(), g.stream);
    return group_step_once(g, false);
}

// ------------------------------------------------------------- validation

static int check_finite(double x, const char *what)
{
    if (!std::isfinite(x)) return fail(SOL_EINVAL, "%s is not finite", what);
    return SOL_OK;
}

static int validate(const sol_grid *g, const sol_alloy *a, const sol_bcs *b, const sol_numerics *n)
{
    if (!g || !a || !b || !n) return fail(SOL_EINVAL, "NULL argument");
    if (g->dim != 2 && g->dim != 3) return fail(SOL_EINVAL, "dim must be 2 or 3 (got %d)", g->dim);
    if (g->nx < 2 || g->ny < 1) return fail(SOL_EINVAL, "need nx >= 2 and ny >= 1 (got %d, %d)", g->nx, g->ny);
    if (g->dim == 3 && g->nz < 1) return fail(SOL_EINVAL, "need nz >= 1 in 3D");
    if (g->dim == 2 && g->nz != 1) return fail(SOL_EINVAL, "2D grids need nz = 1");
    const double cells = (double)g->nx * g->ny * (g->dim == 3 ? g->nz : 1);
    if (cells * 7.0 > 2.0e9) return fail(SOL_EINVAL, "grid too large for 32-bit indices");
    if (!(g->lx > 0) || !(g->ly > 0) || (g->dim == 3 && !(g->lz > 0)))
        return fail(SOL_EINVAL, "domain lengths must be > 0");
    const double v[] = {a->rho, a->mu, a->cp, a->k, a->latent, a->beta_T, a->beta_C, a->lambda2, a->T_m,
                        a->m_sp, a->k_p, a->C_e, a->T_ref, a->C_ref, a->g, a->D_l, a->darcy_eps};
    for (double x : v) RCHK(check_finite(x, "alloy constant"));
    if (!(a->rho > 0) || !(a->mu > 0) || !(a->cp > 0) || !(a->k > 0) || !(a->latent > 0))
        return fail(SOL_EINVAL, "rho, mu, cp, k, latent must be > 0");
    if (!(a->lambda2 > 0)) return fail(SOL_EINVAL, "lambda2 must be > 0");
    if (!(a->k_p > 0 && a->k_p < 1)) return fail(SOL_EINVAL, "k_p must lie in (0,1)");
    if (!(a->m_sp < 0)) return fail(SOL_EINVAL, "liquidus slope m_sp must be < 0");
    if (!(a->C_e > 0)) return fail(SOL_EINVAL, "C_e must be > 0");
    if (!(a->D_l >= 0)) return fail(SOL_EINVAL, "liquid diffusivity D_l must be >= 0");
    if (!(a->darcy_eps >= 0)) return fail(SOL_EINVAL, "darcy_eps must be >= 0");
    if (a->g < 0) return fail(SOL_EINVAL, "g must be >= 0");
    const int nf = g->dim == 3 ? 6 : 4;
    for (int f = 0; f < 6; ++f) {
        const sol_face_bc &fb = b->face[f];
        if (f >= nf) continue;
        if (fb.thermal < 0 || fb.thermal > 2) return fail(SOL_EINVAL, "face %d: bad thermal type", f);
        if (fb.velocity < 0 || fb.velocity > 1) return fail(SOL_EINVAL, "face %d: bad velocity type", f);
        if (fb.thermal == 1 && !(fb.h > 0 && std::isfinite(fb.h) && std::isfinite(fb.T_ext)))
            return fail(SOL_EINVAL, "face %d: Robin wall needs h > 0 and finite T_ext", f);
        if (fb.thermal == 2 && !(std::isfinite(fb.T0) && std::isfinite(fb.b)))
            return fail(SOL_EINVAL, "face %d: prescribed wall temperature needs finite T0, b", f);
    }
    if (!(n->dt > 0) || !std::isfinite(n->dt)) return fail(SOL_EINVAL, "dt must be > 0");
    if (!(n->tol_p > 0 && n->tol_p < 1) || !(n->tol_t > 0 && n->tol_t < 1))
        return fail(SOL_EINVAL, "tolerances must lie in (0,1)");
    if (n->max_iter < 1) return fail(SOL_EINVAL, "max_iter must be >= 1");
    if (n->precision != SOL_PRECISION_FP64 && n->precision != SOL_PRECISION_MIXED)
        return fail(SOL_EINVAL, "precision must be SOL_PRECISION_FP64 or SOL_PRECISION_MIXED");
    return SOL_OK;
}

static void make_phys(const sol_handle &h, Phys &P)
{
    std::memset(&P, 0, sizeof(P));
    const Sizes &z = h.z;
    P.dim = z.dim; P.nx = z.nx; P.ny = z.ny; P.nz = z.nz;
    P.ncell = z.ncell;
    for (int s = 0; s < NSYS; ++s) {
        P.nsys[s] = z.nsys[s];
        for (int a = 0; a < 3; ++a) P.sdim[s][a] = z.sdim[s][a];
    }
    const double L[3] = {h.grid.lx, h.grid.ly, z.dim == 3 ? h.grid.lz : 1.0};
    const int N[3] = {z.nx, z.ny, z.nz};
    for (int a = 0; a < 3; ++a) {
        P.h[a] = L[a] / N[a];
        P.ih[a] = 1.0 / P.h[a];
        P.ih2[a] = 1.0 / (P.h[a] * P.h[a]);
    }
    const sol_alloy &a = h.al;
    P.rho = a.rho; P.mu = a.mu; P.nu = a.mu / a.rho;
    P.dt = h.num.dt; P.idt = 1.0 / h.num.dt;
    P.alpha = a.k / (a.rho * a.cp);
    P.lam = a.latent / a.cp;
    P.kp = a.k_p; P.Tm = a.T_m; P.msp = a.m_sp; P.Ce = a.C_e;
    P.Tref = a.T_ref; P.Cref = a.C_ref; P.grav = a.g;
    P.betaT = a.beta_T; P.betaC = a.beta_C; P.lambda2 = a.lambda2; P.eps = a.darcy_eps;
    P.rcp = a.rho * a.cp; P.kcond = a.k;
    P.Dl = a.D_l;
    P.gfloor = std::cbrt(a.darcy_eps);
    P.mom1 = h.momentum == SOL_MOMENTUM_MINIMAL ? 1 : 0;
    for (int f = 0; f < 6; ++f) {
        const sol_face_bc &fb = h.bcs.face[f];
        const bool used = f < 2 * z.dim;
        P.thermal[f] = used ? fb.thermal : 0;
        P.slip[f] = used ? fb.velocity : 0;
        P.hc[f] = fb.h; P.Text[f] = fb.T_ext; P.Tw0[f] = fb.T0; P.Tramp[f] = fb.b;
    }
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *sol_last_error(void) { return g_err.c_str(); }
const char *sol_version(void) { return "solidify-mi355x 0.1 (gfx950)"; }

int sol_footprint_bytes(const sol_grid *grid, const sol_numerics *num, size_t *out)
{
    if (!grid || !num || !out) return fail(SOL_EINVAL, "NULL argument");
    if ((grid->dim != 2 && grid->dim != 3) || grid->nx < 2 || grid->ny < 1 || (grid->dim == 3 && grid->nz < 1))
        return fail(SOL_EINVAL, "bad grid");
    Sizes z;
    compute_sizes(*grid, z);
    *out = footprint(z, num->precision);
    return SOL_OK;
}

static int alloc_case(sol_handle *h)
{
    const Sizes &z = h->z;
    Mem &m = h->mem;
    m.reserve(footprint(z, h->num.precision));
    const size_t D = sizeof(double);
    CaseDev &d = h->cd;
    std::memset(&d, 0, sizeof(d));
    make_phys(*h, d.ph);
    auto dal = [&](size_t n) { return (double *)m.get(std::max<size_t>(n, 1) * D); };
    // face arrays: one block per set, components back to back
    size_t nf[3];
    for (int s = 0; s < 3; ++s) nf[s] = std::max(z.nsys[s], 1);
    const size_t nft = nf[0] + nf[1] + nf[2];
    double *fu = dal(nft), *fs = dal(nft), *fn = dal(nft), *fp = dal(nft), *fp2 = dal(nft);
    if (!fu || !fs || !fn || !fp || !fp2) return fail(SOL_ENOMEM, "device allocation failed");
    d.u = fu; d.v = fu + nf[0]; d.w = fu + nf[0] + nf[1];
    d.us[0] = fs; d.us[1] = fs + nf[0]; d.us[2] = fs + nf[0] + nf[1];
    d.un[0] = fn; d.un[1] = fn + nf[0]; d.un[2] = fn + nf[0] + nf[1];
    d.usprev[0] = fp; d.usprev[1] = fp + nf[0]; d.usprev[2] = fp + nf[0] + nf[1];
    d.usprev2[0] = fp2; d.usprev2[1] = fp2 + nf[0]; d.usprev2[2] = fp2 + nf[0] + nf[1];
    double **cellf[] = {&d.p,     &d.T,     &d.C,     &d.gl,       &d.Cl,     &d.Cs,      &d.phi,
                        &d.Cnew,  &d.Tstar, &d.Tprev, &d.phiprev, &d.Tprev2, &d.phiprev2};
    for (double **pp : cellf) if (!(*pp = dal(z.ncell))) return fail(SOL_ENOMEM, "device allocation failed");
    for (int s = 0; s < NSYS; ++s) {
        const size_t n = std::max(z.nsys[s], 1);
        d.A[s] = dal(z.nd * n);
        d.b[s] = dal(n);
        d.minv[s] = dal(n);
        if (!d.A[s] || !d.b[s] || !d.minv[s]) return fail(SOL_ENOMEM, "device allocation failed");
        if (s != SP && s != SC) {
            d.Ac[s] = dal(z.nd * n);
            if (!d.Ac[s]) return fail(SOL_ENOMEM, "device allocation failed");
        }
    }
    for (int w = 0; w < 3; ++w)
        for (int k = 0; k < NWORK; ++k)
            if (!(h->work[w][k] = dal(z.maxn))) return fail(SOL_ENOMEM, "device allocation failed");
    if (h->num.precision == SOL_PRECISION_MIXED) {
        auto fal = [&](size_t n) { return (float *)m.get(std::max<size_t>(n, 1) * sizeof(float)); };
        for (int s = 0; s < NSYS; ++s) {
            const size_t n = std::max(z.nsys[s], 1);
            d.A32[s] = fal(z.nd * n);
            d.minv32[s] = fal(n);
            if (!d.A32[s] || !d.minv32[s]) return fail(SOL_ENOMEM, "device allocation failed");
        }
        for (int w = 0; w < 3; ++w)
            for (int k = 0; k < NWORK32; ++k)
                if (!(h->work32[w][k] = fal(z.maxn))) return fail(SOL_ENOMEM, "device allocation failed");
    }
    {
        // pressure multigrid hierarchy: level 0 is the pressure system itself
        MGDims md;
        mg_dims(z, md);
        const bool mixed = h->num.precision == SOL_PRECISION_MIXED;
        auto fal = [&](size_t n) { return (float *)m.get(std::max<size_t>(n, 1) * sizeof(float)); };
        h->mg_nlev = md.nlev;
        h->mg_nglob = md.nglob;
        h->mg_nbig = md.nbig;
        for (int l = 0; l < md.nlev; ++l) {
            MLevel L;
            std::memset(&L, 0, sizeof(L));
            L.n = md.n[l];
            L.nx = md.d[l][0];
            L.ny = md.d[l][1];
            L.nz = md.d[l][2];
            if (l + 1 < md.nlev) {
                L.cn = md.n[l + 1];
                L.cnx = md.d[l + 1][0];
                L.cny = md.d[l + 1][1];
                L.cnz = md.d[l + 1][2];
            } else {
                L.cn = 0;
                L.cnx = L.cny = L.cnz = 1;
            }
            // level 0: tiles of the kernels with partial sums (set with the
            // tuned size by mg_upload); levels >= 1: one thread per child
            L.cpt = l == 0 ? TILE : TILE >> z.dim;
            L.ntile = L.cn ? ceil_div(L.cn, L.cpt) : 0;
            L.sc = 1 << l;
            L.n0[0] = z.nx;
            L.n0[1] = z.ny;
            L.n0[2] = z.nz;
            for (int a = 0; a < 3; ++a) L.ih2[a] = d.ph.ih2[a];
            MLevel L32 = L;
            if (l == 0) {
                L.minv = d.minv[SP];
                L32.minv = d.minv32[SP];
                if (z.dim == 2) {
                    // the level-0 pre-smoothed value (two sweeps in 2D)
                    if (!(L.xs = dal(L.n))) return fail(SOL_ENOMEM, "device allocation failed");
                    if (mixed && !(L32.xs = fal(L.n))) return fail(SOL_ENOMEM, "device allocation failed");
                }
            } else {
                const size_t n = L.n;
                double *mi = dal(n), *bl = dal(n), *el = dal(n), *xl = dal(n);
                if (!mi || !bl || !el || !xl) return fail(SOL_ENOMEM, "device allocation failed");
                L.minv = mi; L.b = bl; L.e = el; L.xs = xl;
                if (mixed) {
                    float *mi32 = fal(n), *b32 = fal(n), *e32 = fal(n), *x32 = fal(n);
                    if (!mi32 || !b32 || !e32 || !x32) return fail(SOL_ENOMEM, "device allocation failed");
                    L32.minv = mi32; L32.b = b32; L32.e = e32; L32.xs = x32;
                }
            }
            if (l == md.nglob) {
                // the elimination runs in FP64 (set-up only); the product of
                // every solve reads the FP32 copy
                const size_t n2 = (size_t)L.n * L.n;
                h->mg_p64 = dal(n2);
                h->mg_pwork = dal(mg_gj_work(L.n));
                float *P32 = fal(n2);
                if (!h->mg_p64 || !h->mg_pwork || !P32) return fail(SOL_ENOMEM, "device allocation failed");
                L.pinv = P32;
                L32.pinv = P32;
            }
            if (md.nbig && l == md.nbig) {
                const size_t n2 = (size_t)L.n * L.n;
                h->mg_pbig64 = dal(n2);
                h->mg_pbigwork = dal(mg_gj_work(L.n));
                float *P32 = fal(n2);
                if (!h->mg_pbig64 || !h->mg_pbigwork || !P32) return fail(SOL_ENOMEM, "device allocation failed");
                L.pinv = P32;
                L32.pinv = P32;
            }
            h->mg_h[l] = L;
            h->mg32_h[l] = L32;
        }
        h->mg_d = (MLevel *)m.get(sizeof(MLevel) * MG_MAXLEV);
        if (!h->mg_d) return fail(SOL_ENOMEM, "device allocation failed");
        if (mixed) {
            h->mg32_d = (MLevel *)m.get(sizeof(MLevel) * MG_MAXLEV);
            if (!h->mg32_d) return fail(SOL_ENOMEM, "device allocation failed");
        }
    }
    d.red_part = dal((size_t)z.ntile_cell * 4);
    d.red_cnt = (uint32_t *)m.get(256);
    d.step = (int64_t *)m.get(256);
    if (!d.red_part || !d.red_cnt || !d.step) return fail(SOL_ENOMEM, "device allocation failed");
    d.hist = d.step + 1;                 // same 256-byte block, zeroed with it
    d.ntile_cell = z.ntile_cell;
    return SOL_OK;
}

static int init_state(sol_handle *h)
{
    CaseDev &d = h->cd;
    hipStream_t s = h->stream;
    const Sizes &z = h->z;
    const int nf = std::max(z.nsys[0], 1) + std::max(z.nsys[1], 1) + std::max(z.nsys[2], 1);
    launch_fill(d.u, 0.0, nf, s);
    launch_fill(d.us[0], 0.0, nf, s);
    launch_fill(d.un[0], 0.0, nf, s);
    launch_fill(d.usprev[0], 0.0, nf, s);
    launch_fill(d.usprev2[0], 0.0, nf, s);
    launch_fill(d.p, 0.0, z.ncell, s);
    launch_fill(d.T, h->al.T_ref, z.ncell, s);
    launch_fill(d.C, h->al.C_ref, z.ncell, s);
    launch_fill(d.gl, 1.0, z.ncell, s);
    launch_fill(d.Cl, h->al.C_ref, z.ncell, s);
    launch_fill(d.Cs, 0.0, z.ncell, s);
    launch_fill(d.phi, 0.0, z.ncell, s);
    launch_fill(d.Cnew, h->al.C_ref, z.ncell, s);
    launch_fill(d.Tstar, h->al.T_ref, z.ncell, s);
    launch_fill(d.Tprev, 0.0, z.ncell, s);
    launch_fill(d.phiprev, 0.0, z.ncell, s);
    launch_fill(d.Tprev2, 0.0, z.ncell, s);
    launch_fill(d.phiprev2, 0.0, z.ncell, s);
    for (int w = 0; w < 3; ++w)
        for (int k = 0; k < NWORK; ++k) launch_fill(h->work[w][k], 0.0, z.maxn, s);
    for (int w = 0; w < 3; ++w)
        for (int k = 0; k < NWORK32; ++k)
            if (h->work32[w][k]) HIPCHK(hipMemsetAsync(h->work32[w][k], 0, sizeof(float) * std::max(z.maxn, 1), s));
    HIPCHK(hipMemsetAsync(d.red_cnt, 0, 256, s));
    HIPCHK(hipMemsetAsync(d.step, 0, 256, s));
    HIPCHK(hipGetLastError());
    return SOL_OK;
}

int sol_create(const sol_grid *grid, const sol_alloy *alloy, const sol_bcs *bcs, const sol_numerics *num,
               const sol_device_ctx *ctx, sol_handle **out)
{
    if (!out) return fail(SOL_EINVAL, "NULL out");
    *out = nullptr;
    RCHK(validate(grid, alloy, bcs, num));
    if (ctx && ((ctx->alloc == nullptr) != (ctx->free == nullptr)))
        return fail(SOL_EINVAL, "ctx->alloc and ctx->free must both be set or both be NULL");
    sol_handle *h = new sol_handle();
    h->grid = *grid;
    if (h->grid.dim == 2) { h->grid.nz = 1; h->grid.lz = 1.0; }
    h->al = *alloy;
    h->bcs = *bcs;
    h->num = *num;
    compute_sizes(h->grid, h->z);
    if (ctx) {
        h->stream = (hipStream_t)ctx->stream;
        if (ctx->alloc) { h->mem.ctx = *ctx; h->mem.has_ctx = true; }
    }
    int rc = alloc_case(h);
    if (rc == SOL_OK) rc = init_state(h);
    if (rc == SOL_OK) rc = group_create({h}, &h->solo);
    if (rc == SOL_OK) {
        Group &g = *h->solo;
        for (int gi = 0; gi < 2; ++gi) launch_asm_const(gi ? 3 : 2, g.cases_d, g.t_const[gi], g.n_const[gi], h->stream);
        // inverse diagonals of the coarse multigrid levels of the (constant)
        // pressure operator
        const bool mixed = h->num.precision == SOL_PRECISION_MIXED;
        for (int l = 1; l < h->mg_nlev; ++l)
            launch_mg_minv(h->z.dim, h->mg_d, l, h->mg_h[l].n, (double *)h->mg_h[l].minv,
                           mixed ? (float *)h->mg32_h[l].minv : nullptr, h->stream);
        const int L = h->mg_nglob;
        launch_mg_pinv(h->z.dim, h->mg_d, L, h->mg_h[L].n, h->mg_p64, (float *)h->mg_h[L].pinv, h->mg_pwork,
                       h->stream);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
            rc = fail(SOL_EDEVICE, "offline assembly failed");
    }
    if (rc != SOL_OK) {
        group_free(h->solo);
        h->mem.release();
        delete h;
        return rc;
    }
    *out = h;
    return SOL_OK;
}

void sol_destroy(sol_handle *h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    group_free(h->solo);
    for (int s = 0; s < NSYS; ++s) {
        if (h->csr_rp[s]) (void)hipFree(h->csr_rp[s]);
        if (h->csr_col[s]) (void)hipFree(h->csr_col[s]);
        if (h->csr_val[s]) (void)hipFree(h->csr_val[s]);
    }
    if (h->csr_cnt) (void)hipFree(h->csr_cnt);
    for (auto &s : h->samples) { (void)hipEventDestroy(s.a); (void)hipEventDestroy(s.b); }
    for (auto e : h->event_pool) (void)hipEventDestroy(e);
    h->mem.release();
    delete h;
}

static double *field_ptr(sol_handle *h, int bit, size_t *n)
{
    const Sizes &z = h->z;
    CaseDev &d = h->cd;
    switch (bit) {
    case 0: *n = z.nsys[0]; return d.u;
    case 1: *n = z.nsys[1]; return d.v;
    case 2: *n = z.nsys[2]; return d.w;
    case 3: *n = z.ncell; return d.p;
    case 4: *n = z.ncell; return d.T;
    case 5: *n = z.ncell; return d.C;
    case 6: *n = z.ncell; return d.gl;
    case 7: *n = z.ncell; return d.Cl;
    case 8: *n = z.ncell; return d.Cs;
    case 9: *n = z.nsys[0]; return d.us[0];
    case 10: *n = z.nsys[1]; return d.us[1];
    case 11: *n = z.nsys[2]; return d.us[2];
    case 12: *n = z.ncell; return d.phi;
    case 13: *n = z.ncell; return d.Tstar;
    }
    *n = 0;
    return nullptr;
}

int sol_write_fields(sol_handle *h, uint32_t mask, const double *const *src)
{
    if (!h || !src) return fail(SOL_EINVAL, "NULL argument");
    if (mask & ~((1u << 9) - 1)) return fail(SOL_EINVAL, "only state fields (SOL_F_U..SOL_F_CS) can be written");
    if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
    for (int bit = 0; bit < 9; ++bit) {
        if (!(mask & (1u << bit))) continue;
        size_t n;
        field_ptr(h, bit, &n);
        if (n && !src[bit]) return fail(SOL_EINVAL, "field %d: NULL source", bit);
        for (size_t i = 0; i < n; ++i)
            if (!std::isfinite(src[bit][i])) return fail(SOL_ENONFINITE, "field %d: non-finite value at %zu", bit, i);
    }
    for (int bit = 0; bit < 9; ++bit) {
        if (!(mask & (1u << bit))) continue;
        size_t n;
        double *d = field_ptr(h, bit, &n);
        if (n) HIPCHK(hipMemcpyAsync(d, src[bit], n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    }
    // the solution history no longer belongs to these fields
    HIPCHK(hipMemcpyAsync(h->cd.hist, h->cd.step, sizeof(int64_t), hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SOL_OK;
}

int sol_read_fields(sol_handle *h, uint32_t mask, double *const *dst)
{
    if (!h || !dst) return fail(SOL_EINVAL, "NULL argument");
    if (mask & ~((1u << SOL_NFIELDS) - 1)) return fail(SOL_EINVAL, "unknown field bits");
    for (int bit = 0; bit < SOL_NFIELDS; ++bit) {
        if (!(mask & (1u << bit))) continue;
        size_t n;
        field_ptr(h, bit, &n);
        if (n && !dst[bit]) return fail(SOL_EINVAL, "field %d: NULL destination", bit);
    }
    for (int bit = 0; bit < SOL_NFIELDS; ++bit) {
        if (!(mask & (1u << bit))) continue;
        size_t n;
        double *d = field_ptr(h, bit, &n);
        if (n) HIPCHK(hipMemcpyAsync(dst[bit], d, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return SOL_OK;
}

int sol_system_size(const sol_handle *h, int32_t system, int32_t *rows, int32_t *nnz)
{
    if (!h || !rows || !nnz) return fail(SOL_EINVAL, "NULL argument");
    if (system < 0 || system >= NSYS) return fail(SOL_EINVAL, "bad system %d", system);
    const Sizes &z = h->z;
    const int *d = z.sdim[system];
    const int64_t n = (int64_t)d[0] * d[1] * d[2];
    int64_t k = n;
    if (n) {
        k += 2 * ((int64_t)(d[0] - 1) * d[1] * d[2] + (int64_t)d[0] * (d[1] - 1) * d[2]);
        if (z.dim == 3) k += 2 * (int64_t)d[0] * d[1] * (d[2] - 1);
    }
    *rows = (int32_t)n;
    *nnz = (int32_t)k;
    return SOL_OK;
}

int sol_assemble(sol_handle *h, uint32_t mask)
{
    if (!h) return fail(SOL_EINVAL, "NULL handle");
    if (mask & ~((1u << NSYS) - 1)) return fail(SOL_EINVAL, "unknown system bits");
    if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
    Group &g = *h->solo;
    hipStream_t s = h->stream;
    const int gi = h->z.dim == 3 ? 1 : 0;
    const int dim = h->z.dim;
    const int fwd = h->assembly == SOL_ASSEMBLY_FORWARD;
    if (mask & 7u) launch_asm_momentum(dim, g.cases_d, g.t_mom[gi], g.n_mom[gi], s, fwd);
    if (mask & (1u << SP)) {
        launch_div_rhs(dim, g.cases_d, g.t_cell[gi], g.n_cell[gi], 0, s);
        launch_case_mean(g.cases_d, g.cidx_d, 1, s);
        launch_sub_mean(g.cases_d, g.t_cell[gi], g.n_cell[gi], s);
    }
    if (mask & ((1u << SC) | (1u << ST))) launch_asm_transport(dim, g.cases_d, g.t_cell[gi], g.n_cell[gi], 0, s, fwd);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return SOL_OK;
}

int sol_read_matrix(sol_handle *h, int32_t system, int32_t *row_ptr, int32_t *col_idx, double *val, double *rhs)
{
    if (!h || !row_ptr || !col_idx || !val || !rhs) return fail(SOL_EINVAL, "NULL argument");
    if (system < 0 || system >= NSYS) return fail(SOL_EINVAL, "bad system %d", system);
    int32_t n, nnz;
    RCHK(sol_system_size(h, system, &n, &nnz));
    if (n == 0) { row_ptr[0] = 0; return SOL_OK; }
    const bool build = h->csr_rp[system] == nullptr;
    if (build) {
        if (!h->csr_cnt) HIPCHK(hipMalloc(&h->csr_cnt, sizeof(int32_t) * h->z.maxn));
        HIPCHK(hipMalloc(&h->csr_rp[system], sizeof(int32_t) * (n + 1)));
        HIPCHK(hipMalloc(&h->csr_col[system], sizeof(int32_t) * nnz));
        HIPCHK(hipMalloc(&h->csr_val[system], sizeof(double) * nnz));
    }
    // device descriptor of this case (solo group entry 0)
    launch_csr(h->z.dim, h->solo->cases_d, system, n, h->csr_cnt, h->csr_rp[system], h->csr_col[system],
               h->csr_val[system], build ? 1 : 0, h->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(row_ptr, h->csr_rp[system], sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(col_idx, h->csr_col[system], sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(val, h->csr_val[system], sizeof(double) * nnz, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(rhs, h->cd.b[system], sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SOL_OK;
}

// ------------------------------------------------ allocation-free export
// Device scratch of sol_read_matrix_noalloc: one array per GPU the library
// runs on, held until the process ends.  On the host the array's name is a
// stand-in, not device memory: host code never passes it to a kernel or a
// copy, it uses the device address hipGetSymbolAddress returns, looked up
// once per device with that device current and kept per device.
static __device__ __align__(256) unsigned char scratch[SOL_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_ptr;

static int scratch_ptr(unsigned char **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SOL_EDEVICE, "device scratch of device %d has no address", dev);
        it = g_scratch_ptr.emplace(dev, (unsigned char *)p).first;
    }
    *out = it->second;
    return SOL_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Layout of the scratch: row counts (rows ints), row_ptr (rows + 1 ints),
// then one block of columns and values; rows go through in blocks whose
// entries fit that block.  Every word a kernel reads was written earlier in
// the same call (counts before the scan, the scan before the fills), so
// nothing is cleared.
int sol_read_matrix_noalloc(sol_handle *h, int32_t system, int32_t *row_ptr, int32_t *col_idx, double *val,
                            double *rhs)
{
    if (!h || !row_ptr || !col_idx || !val || !rhs) return fail(SOL_EINVAL, "NULL argument");
    if (system < 0 || system >= NSYS) return fail(SOL_EINVAL, "bad system %d", system);
    int32_t n, nnz;
    RCHK(sol_system_size(h, system, &n, &nnz));
    if (n == 0) { row_ptr[0] = 0; return SOL_OK; }
    const size_t total = SOL_NOALLOC_SCRATCH_BYTES;
    const size_t pat = align256(sizeof(int32_t) * (size_t)n) + align256(sizeof(int32_t) * ((size_t)n + 1));
    const size_t row_max = (size_t)h->z.nd * (sizeof(int32_t) + sizeof(double));
    if (pat + row_max + 512 > total)
        return fail(SOL_EINVAL, "system %d has %d rows: its CSR row pointers (%zu bytes) do not fit the %zu-byte "
                    "device scratch of the allocation-free export", system, n, pat, total);
    unsigned char *sp = nullptr;
    RCHK(scratch_ptr(&sp));
    int32_t *cnt = (int32_t *)sp;
    int32_t *rp = (int32_t *)(sp + align256(sizeof(int32_t) * (size_t)n));
    const size_t cap = (total - pat - 512) / (sizeof(int32_t) + sizeof(double));     // entries per block
    int32_t *col = (int32_t *)(sp + pat);
    double *vv = (double *)(sp + pat + align256(sizeof(int32_t) * cap));
    hipStream_t st = h->stream;
    const int dim = h->z.dim;
    const CaseDev *cd = h->solo->cases_d;
    launch_csr_pattern(dim, cd, system, n, cnt, rp, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(row_ptr, rp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (row_ptr[n] != nnz) return fail(SOL_EDEVICE, "CSR pattern of system %d: %d entries, expected %d", system,
                                       row_ptr[n], nnz);
    // stream order keeps each block's copies ahead of the next block's fill
    for (int r0 = 0; r0 < n;) {
        const int32_t lim = row_ptr[r0] + (int32_t)std::min<size_t>(cap, (size_t)nnz);
        const int r1 = (int)(std::upper_bound(row_ptr + r0 + 1, row_ptr + n + 1, lim) - row_ptr) - 1;
        const int32_t base = row_ptr[r0];
        const size_t m = (size_t)(row_ptr[r1] - base);
        launch_csr_rows(dim, cd, system, r0, r1, rp, base, col, vv, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(col_idx + base, col, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(val + base, vv, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        r0 = r1;
    }
    HIPCHK(hipMemcpyAsync(rhs, h->cd.b[system], sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return SOL_OK;
}

static int fill_stats(Group &g, int c, sol_step_stats *st, const int64_t *tot)
{
    sol_handle *h = g.cs[c];
    KState ks[NSYS];
    double red[16];
    int64_t step = 0;
    note_dispatch(3);
    HIPCHK(hipMemcpyAsync(ks, g.ks_d + c * NSYS, sizeof(ks), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipMemcpyAsync(red, g.red_d + 16 * c, sizeof(red), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipMemcpyAsync(&step, h->cd.step, sizeof(step), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    std::memset(st, 0, sizeof(*st));
    for (int s = 0; s < NSYS; ++s) {
        if (h->z.nsys[s] == 0) continue;
        st->iters[s] = ks[s].it;
        st->iters_total[s] = tot ? tot[s] : ks[s].it;
        st->rel_resid[s] = ks[s].bb > 0 ? std::sqrt(ks[s].tr2 / ks[s].bb) : 0.0;
        st->sum_resid[s] = ks[s].tsum;
    }
    st->sum_C = red[R_SUMC];
    st->sum_H = red[R_SUMH];
    st->wall_flux = red[R_WALL];
    st->div_star = red[R_DIVSTAR];
    st->div_new = red[R_DIVNEW];
    st->step = step;
    st->redone = h->redone;
    return SOL_OK;
}

// build the larger exact level's inverse of a large grid (once, before its
// first multigrid solve alone) and rebuild the case's own group with it
static int mg_big_prepare(sol_handle *h)
{
    if (h->mg_nbig <= 0 || h->mg_big_ready || h->precond != SOL_PRECOND_MG) return SOL_OK;
    const int L = h->mg_nbig;
    launch_mg_pinv(h->z.dim, h->mg_d, L, h->mg_h[L].n, h->mg_pbig64, (float *)h->mg_h[L].pinv, h->mg_pbigwork,
                   h->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
        return fail(SOL_EDEVICE, "multigrid set-up failed");
    h->mg_big_ready = true;
    group_free(h->solo);
    h->solo = nullptr;
    return group_create({h}, &h->solo);
}

int sol_step(sol_handle *h, int32_t nsteps, sol_step_stats *stats)
{
    if (!h) return fail(SOL_EINVAL, "NULL handle");
    if (nsteps < 0) return fail(SOL_EINVAL, "nsteps must be >= 0");
    if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
    if (nsteps > 0) RCHK(mg_big_prepare(h));
    Group &g = *h->solo;
    g.timer = h->timing ? h : nullptr;
    g.use_graph = h->opt_graph;
    int64_t tot[NSYS] = {};
    for (int k = 0; k < nsteps; ++k) {
        int rc = group_step(g);
        if (rc != SOL_OK) {
            // a failed step leaves partial solutions in the step buffers
            launch_hist_reset(g.cases_d, (int)g.cs.size(), g.stream);
            (void)hipStreamSynchronize(h->stream);
            return rc;
        }
        for (int s = 0; s < NSYS; ++s) tot[s] += h->last_iters[s];
        if (g.timer) {
            HIPCHK(hipStreamSynchronize(h->stream));
            collect_samples(g, g.ks_h[0]);
        }
    }
    if (stats) RCHK(fill_stats(g, 0, stats, tot));
    else HIPCHK(hipStreamSynchronize(h->stream));
    return SOL_OK;
}

int sol_dispatch_count(int64_t *count)
{
    if (!count) return fail(SOL_EINVAL, "NULL argument");
    *count = (int64_t)dispatch_count();
    return SOL_OK;
}

int sol_set_timing(sol_handle *h, int32_t enable)
{
    if (!h) return fail(SOL_EINVAL, "NULL handle");
    h->timing = enable != 0;
    for (auto &t : h->tacc) t = TAcc();
    return SOL_OK;
}

int sol_get_timing(sol_handle *h, int32_t kclass, int64_t *launches, double *total_ms, double *bytes)
{
    if (!h || !launches || !total_ms || !bytes) return fail(SOL_EINVAL, "NULL argument");
    if (kclass < 0 || kclass >= SOL_NKCLASS) return fail(SOL_EINVAL, "bad kernel class");
    *launches = h->tacc[kclass].n;
    *total_ms = h->tacc[kclass].ms;
    *bytes = h->tacc[kclass].bytes;
    return SOL_OK;
}

int sol_set_option(sol_handle *h, int32_t option, int64_t value)
{
    if (!h) return fail(SOL_EINVAL, "NULL handle");
    switch (option) {
    case SOL_OPT_GRAPH: h->opt_graph = value != 0; return SOL_OK;
    case SOL_OPT_PRECOND: {
        if (value != SOL_PRECOND_JACOBI && value != SOL_PRECOND_MG)
            return fail(SOL_EINVAL, "unknown preconditioner %lld", (long long)value);
        if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
        if (h->precond == (int)value) return SOL_OK;
        (void)hipStreamSynchronize(h->stream);
        h->precond = (int)value;
        group_free(h->solo);
        h->solo = nullptr;
        return group_create({h}, &h->solo);
    }
    case SOL_OPT_TPRECOND: {
        if (value != SOL_TPRECOND_JACOBI && value != SOL_TPRECOND_JACOBI2 && value != SOL_TPRECOND_AUTO)
            return fail(SOL_EINVAL, "unknown transport preconditioner %lld", (long long)value);
        if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
        if (h->tprecond == (int)value) return SOL_OK;
        (void)hipStreamSynchronize(h->stream);
        h->tprecond = (int)value;
        group_free(h->solo);
        h->solo = nullptr;
        return group_create({h}, &h->solo);
    }
    case SOL_OPT_ASSEMBLY: {
        if (value != SOL_ASSEMBLY_STENCIL && value != SOL_ASSEMBLY_FORWARD)
            return fail(SOL_EINVAL, "unknown assembly route %lld", (long long)value);
        if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
        h->assembly = (int)value;
        return SOL_OK;
    }
    case SOL_OPT_MG_FUSE: {
        if (value != 0 && value != 1) return fail(SOL_EINVAL, "SOL_OPT_MG_FUSE takes 0 or 1");
        if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
        if (h->mg_fuse == (value != 0)) return SOL_OK;
        (void)hipStreamSynchronize(h->stream);
        h->mg_fuse = value != 0;
        group_free(h->solo);
        h->solo = nullptr;
        return group_create({h}, &h->solo);
    }
    case SOL_OPT_MOMENTUM: {
        if (value != SOL_MOMENTUM_PLAIN && value != SOL_MOMENTUM_MINIMAL)
            return fail(SOL_EINVAL, "unknown momentum form %lld", (long long)value);
        if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
        if (h->momentum == (int)value) return SOL_OK;
        (void)hipStreamSynchronize(h->stream);
        h->momentum = (int)value;
        h->cd.ph.mom1 = h->momentum == SOL_MOMENTUM_MINIMAL ? 1 : 0;
        // the case's groups hold a device copy of its Phys
        group_free(h->solo);
        h->solo = nullptr;
        return group_create({h}, &h->solo);
    }
    }
    return fail(SOL_EINVAL, "unknown option %d", option);
}

// time iterations of the pressure solve (FP32 inner solve for mixed
// precision) with the current tiles; never converges (tol 0).  The rhs is
// mean-free so that the singular Neumann system stays consistent.
static int time_pressure(sol_handle *h, double *ms_per_iter)
{
    Group &g = *h->solo;
    Phase &P = g.ph[1];
    const bool fp32 = g.precision == SOL_PRECISION_MIXED;
    JobSet &S = fp32 ? P.inner : P.main;
    if (S.jobs.empty()) return fail(SOL_EINVAL, "no pressure system to tune");
    const KJob &J = S.jobs[0];
    launch_tune_rhs((void *)J.b, fp32 ? 1 : 0, J.n, g.stream);
    const double zero = 0.0;
    const int running = K_RUNNING;
    HIPCHK(hipMemcpy((char *)J.st + offsetof(KState, tol2), &zero, sizeof(zero), hipMemcpyHostToDevice));
    if (fp32)
        HIPCHK(hipMemcpy((char *)J.partner + offsetof(KState, status), &running, sizeof(running), hipMemcpyHostToDevice));
    // Multigrid reduces the residual about tenfold per iteration: a run
    // must stay far above rounding, or a breakdown restarts the solve and
    // the launches after it time as no-ops (14 iterations did at 500x300
    // and picked a tile size that made the step 17 % slower).  So three
    // short runs from a fresh start, the fastest taken.
    const bool mg = P.kind == K_MGCG;
    const int warm = mg ? 1 : 8, timed_its = mg ? 6 : 48, runs = mg ? 3 : 1;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    float best = 0.f;
    for (int run = 0; run < runs; ++run) {
        RCHK(start_solves(g, P, S, fp32 ? 1 : 0, 0, 0));
        for (int k = 0; k < warm; ++k)
            for (const Stage &st : S.iter) RCHK(launch_stage(g, S, st, fp32 ? 1 : 0, k));
        HIPCHK(hipEventRecord(a, g.stream));
        for (int k = warm; k < warm + timed_its; ++k)
            for (const Stage &st : S.iter) RCHK(launch_stage(g, S, st, fp32 ? 1 : 0, k));
        HIPCHK(hipEventRecord(b, g.stream));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        if (run == 0 || ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    HIPCHK(hipGetLastError());
    *ms_per_iter = best / timed_its;
    return SOL_OK;
}

int sol_autotune(sol_handle *h, int32_t *rows_per_tile_out)
{
    if (!h) return fail(SOL_EINVAL, "NULL handle");
    if (h->batch) return fail(SOL_EBUSY, "handle is part of a batch");
    RCHK(mg_big_prepare(h));
    const int n = h->z.nsys[SP], nd = h->z.nd;
    const int cls = size_class(n, nd);
    const bool mg = h->precond == SOL_PRECOND_MG;
    std::map<int, int> &table = mg ? g_tuned_cpt : g_tuned_rpt;
    const int units = mg ? h->mg_h[0].cn : n;      // what one tile covers a part of
    std::vector<int> cand = mg ? std::vector<int>{256, 512, 1024, 2048} : std::vector<int>{256, 512, 1024, 2048, 4096};
    int best = -1;
    double best_ms = 1e300;
    int rc = SOL_OK;
    for (int c : cand) {
        const int nt = ceil_div(units, c);
        if (nt > 8192 || (c > 256 && nt < 8)) continue;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            table[cls] = c;
        }
        group_free(h->solo);
        h->solo = nullptr;
        rc = group_create({h}, &h->solo);
        if (rc != SOL_OK) break;
        double ms = 0.0;
        rc = time_pressure(h, &ms);
        if (rc != SOL_OK) break;
        if (ms < best_ms) { best_ms = ms; best = c; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (best > 0) table[cls] = best;
        else table.erase(cls);
    }
    (void)hipStreamSynchronize(h->stream);
    group_free(h->solo);
    h->solo = nullptr;
    const int rc2 = group_create({h}, &h->solo);
    if (rc != SOL_OK) return rc;
    if (rc2 != SOL_OK) return rc2;
    if (rows_per_tile_out) *rows_per_tile_out = best;
    return SOL_OK;
}

// ------------------------------------------------------------------ batches

struct sol_batch {
    std::vector<sol_handle *> cs;
    Group *g = nullptr;                  // group over the currently active cases
    std::vector<int> active;
};

int sol_batch_create(sol_handle *const *cases, int32_t n, sol_batch **out)
{
    if (!cases || !out || n < 1) return fail(SOL_EINVAL, "bad batch arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!cases[i]) return fail(SOL_EINVAL, "NULL handle %d", i);
        if (cases[i]->batch) return fail(SOL_EBUSY, "handle %d already in a batch", i);
        if (cases[i]->stream != cases[0]->stream) return fail(SOL_EINVAL, "handles must share one stream");
        if (cases[i]->num.precision != cases[0]->num.precision)
            return fail(SOL_EINVAL, "handles of one batch must share one precision");
        if (cases[i]->precond != cases[0]->precond)
            return fail(SOL_EINVAL, "handles of one batch must share one pressure preconditioner");
        if (cases[i]->tprecond != cases[0]->tprecond)
            return fail(SOL_EINVAL, "handles of one batch must share one transport preconditioner");
        if (cases[i]->assembly != cases[0]->assembly)
            return fail(SOL_EINVAL, "handles of one batch must share one assembly route");
        for (int j = 0; j < i; ++j)
            if (cases[j] == cases[i]) return fail(SOL_EINVAL, "handle %d given twice", i);
    }
    sol_batch *b = new sol_batch();
    b->cs.assign(cases, cases + n);
    for (auto *h : b->cs) h->batch = b;
    *out = b;
    return SOL_OK;
}

void sol_batch_destroy(sol_batch *b)
{
    if (!b) return;
    if (!b->cs.empty()) (void)hipStreamSynchronize(b->cs[0]->stream);
    group_free(b->g);
    for (auto *h : b->cs) h->batch = nullptr;
    delete b;
}

int sol_batch_step(sol_batch *b, const int32_t *nsteps, sol_step_stats *stats)
{
    if (!b || !nsteps) return fail(SOL_EINVAL, "NULL argument");
    const int n = (int)b->cs.size();
    int mx = 0;
    for (int i = 0; i < n; ++i) {
        if (nsteps[i] < 0) return fail(SOL_EINVAL, "nsteps[%d] < 0", i);
        mx = std::max(mx, (int)nsteps[i]);
    }
    std::vector<int64_t> tot((size_t)n * NSYS, 0);
    for (int k = 0; k < mx; ++k) {
        std::vector<int> act;
        for (int i = 0; i < n; ++i) if (nsteps[i] > k) act.push_back(i);
        if (act != b->active || !b->g) {
            if (b->g) { (void)hipStreamSynchronize(b->cs[0]->stream); group_free(b->g); b->g = nullptr; }
            std::vector<sol_handle *> hs;
            for (int i : act) hs.push_back(b->cs[i]);
            RCHK(group_create(hs, &b->g));
            b->active = act;
        }
        b->g->timer = nullptr;
        b->g->use_graph = b->cs[0]->opt_graph;
        int rc = group_step(*b->g);
        if (rc != SOL_OK) {
            launch_hist_reset(b->g->cases_d, (int)b->g->cs.size(), b->g->stream);
            (void)hipStreamSynchronize(b->cs[0]->stream);
            return rc;
        }
        for (size_t a = 0; a < act.size(); ++a)
            for (int s = 0; s < NSYS; ++s) tot[(size_t)act[a] * NSYS + s] += b->cs[act[a]]->last_iters[s];
    }
    if (stats && b->g) {
        for (size_t a = 0; a < b->active.size(); ++a)
            RCHK(fill_stats(*b->g, (int)a, &stats[b->active[a]], &tot[(size_t)b->active[a] * NSYS]));
    }
    HIPCHK(hipStreamSynchronize(b->cs[0]->stream));
    return SOL_OK;
}

}  // extern "C"
