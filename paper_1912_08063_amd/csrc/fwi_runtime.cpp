// fwi_runtime.cpp -- host runtime and C ABI of libfwi.so.
//
// Validates arguments on the host, lays the caller's workspace out into
// fields and tables, and drives the time loops: the forward sweep (Eq. 3 with
// sponge), the misfit (Eq. 1), and the adjoint sweep with the imaging
// condition, recomputing forward levels from checkpoints (every-k segments or
// a binomial revolve schedule).  Every shot of a call is one job of a job
// table, so each launch advances all shots at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "fwi.h"
#include "fwi_internal.h"
#include "revolve.h"

namespace fwi {
void launch_step(int ndim, int M, int nw, bool adj, const Job *jobs, const int *prefix,
                 int njobs, int step, int ttiles, int gblocks, int remap, const LevelMap &lm,
                 hipStream_t st);
void launch_prep_kappa(const float *v, float *kappa, int M, int gy, int nz, int ny, int nx,
                       int pitch, int nya, int nb, int nzm, int nym, int nxm, int64_t total,
                       float dt_dx, hipStream_t st);
void launch_fill(float *p, int64_t n, float val, hipStream_t st);
void launch_zero_frames(float *p, int64_t nfields, int64_t fstride, int nya, int pitch, int M,
                        int gy, int nz, int ny, int nx, hipStream_t st);
void launch_snapshot(const Job *jobs, int njobs, int64_t fstride, int slot, int time, int dir,
                     int mask, const LevelMap &lm, hipStream_t st);
void launch_gather(const Job *jobs, const int *gprefix, int njobs, int gblocks, int threads,
                   int step, const LevelMap &lm, hipStream_t st);
void launch_adj_inject(const Job *jobs, const int *gprefix, int njobs, int gblocks, int threads,
                       int step, hipStream_t st);
int misfit_partials();
void launch_misfit(const float *d, const float *obs, float *res, int64_t n, double *partial,
                   double *out, hipStream_t st);
void launch_fold(int ndim, const Job *jobs, int njobs, int M, int gy, int nz, int ny, int nx,
                 int nb, int nzm, int nym, int nxm, float *tmp1, float *tmp2, const float *v,
                 float *dv, hipStream_t st);
int vstats_blocks();
int step_blocks_per_cu(int ndim, int M, int nw, bool adj);
void launch_vstats(const float *v, int64_t n, float *partial, hipStream_t st);
void launch_nonfinite_level(const Job *jobs, int njobs, int L, float *partial, hipStream_t st);
void launch_assemble(const AssembleArgs &a, Job *table, int *prefix, int32_t *levels,
                     hipStream_t st);
int multi2d_steps();
void multi2d_tile(int M, int *ox, int *oz);
void launch_step2d_multi(int M, const Job *jobs, int njobs, int tiles_per_job, int ntxm,
                         int step, int kk, bool record, hipStream_t st);
int scratch_address(void **ptr);
void launch_stream_probe(const float *a, const float *b, const float *c, float *o, int64_t n,
                         int variant, hipStream_t st);
void launch_tile_probe(const float *cur, const float *prv, const float *kap, float *out, int nz,
                       int ny, int nx, int pitch, int zc, int mode, hipStream_t st);
}  // namespace fwi

using namespace fwi;

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

static int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(FWI_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

// ---------------------------------------------------------------- geometry
namespace {

constexpr uint64_t kAlign = 256;

uint64_t align_up(uint64_t a, uint64_t b) { return (a + b - 1) / b * b; }

struct Geometry {
    int ndim = 0, M = 0, gy = 0;
    int nzm = 1, nym = 1, nxm = 1;   // model grid
    int nb = 0;
    int nz = 1, ny = 1, nx = 1;      // padded grid
    int pitch = 0, nya = 0;
    int64_t plane = 0, fstride = 0;
    int64_t model_cells = 0;
};

int check_problem(const fwi_problem *p)
{
    if (!p) return fail(FWI_EINVAL, "problem is NULL");
    if (p->ndim != 2 && p->ndim != 3) return fail(FWI_EINVAL, "ndim must be 2 or 3");
    for (int a = 0; a < p->ndim; ++a)
        if (p->shape[a] < 1 || p->shape[a] > (1 << 20))
            return fail(FWI_EINVAL, "shape[%d] = %d out of range", a, p->shape[a]);
    if (!(p->dx > 0.f) || !std::isfinite(p->dx)) return fail(FWI_EINVAL, "dx must be > 0");
    if (!(p->dt > 0.f) || !std::isfinite(p->dt)) return fail(FWI_EINVAL, "dt must be > 0");
    if (p->nt < 1) return fail(FWI_EINVAL, "nt must be >= 1");
    if (p->order != 2 && p->order != 4 && p->order != 8 && p->order != 16)
        return fail(FWI_EINVAL, "order must be 2, 4, 8 or 16");
    if (p->nsponge < 0 || p->nsponge > 4096) return fail(FWI_EINVAL, "nsponge out of range");
    if (!std::isfinite(p->eta_max))
        return fail(FWI_EINVAL, "eta_max must be finite (negative: derived from v_max)");
    if (p->nshots < 1) return fail(FWI_EINVAL, "nshots must be >= 1");
    if (p->nrec < 0) return fail(FWI_EINVAL, "nrec must be >= 0");
    return FWI_OK;
}

int make_geometry(const fwi_problem *p, Geometry *g)
{
    int st = check_problem(p);
    if (st) return st;
    g->ndim = p->ndim;
    g->M = p->order / 2;
    g->gy = p->ndim == 3 ? g->M : 0;
    g->nb = p->nsponge;
    g->nzm = p->shape[0];
    g->nym = p->ndim == 3 ? p->shape[1] : 1;
    g->nxm = p->ndim == 3 ? p->shape[2] : p->shape[1];
    g->nz = g->nzm + 2 * g->nb;
    g->ny = p->ndim == 3 ? g->nym + 2 * g->nb : 1;
    g->nx = g->nxm + 2 * g->nb;
    g->pitch = (int)align_up((uint64_t)g->nx + 2 * g->M, 64);
    g->nya = g->ny + 2 * g->gy;
    g->plane = (int64_t)g->nya * g->pitch;
    g->fstride = (int64_t)(g->nz + 2 * g->M) * g->plane;
    g->model_cells = (int64_t)g->nzm * g->nym * g->nxm;
    if (g->fstride > (int64_t(1) << 40)) return fail(FWI_EINVAL, "grid too large");
    // the step kernels address a plane with 32-bit byte offsets
    if (g->plane * (int64_t)sizeof(float) >= (int64_t(1) << 31))
        return fail(FWI_EINVAL, "grid plane too large");
    return FWI_OK;
}

// largest symbol of one axis of the central stencil, S = max_k -(c0 + 2 sum c_m cos(mk))
double max_symbol_scan(int order)
{
    const int M = order / 2;
    double fM = 1;
    for (int i = 2; i <= M; ++i) fM *= i;
    std::vector<double> c(M + 1, 0.0);
    for (int m = 1; m <= M; ++m) {
        double a = 1, b = 1;
        for (int i = 2; i <= M - m; ++i) a *= i;
        for (int i = 2; i <= M + m; ++i) b *= i;
        c[m] = 2.0 * ((m & 1) ? 1.0 : -1.0) * fM * fM / (double(m) * m * a * b);
        c[0] -= 2.0 * c[m];
    }
    double best = 0;
    const int K = 20000;
    for (int i = 0; i <= K; ++i) {
        const double k = M_PI * i / K;
        double s = c[0];
        for (int m = 1; m <= M; ++m) s += 2.0 * c[m] * std::cos(m * k);
        best = std::max(best, -s);
    }
    return best;
}

// The scan above costs about 0.5 ms (80 000 cosines at 8th order); every call
// validates its time step with it, so each order's value is kept after its
// first use (concurrent first uses compute the same value).
double max_symbol(int order)
{
    static std::atomic<double> known[9];
    const int M = order / 2;
    if (M < 1 || M > 8) return max_symbol_scan(order);
    double v = known[M].load(std::memory_order_relaxed);
    if (v <= 0.0) {
        v = max_symbol_scan(order);
        known[M].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Default peak damping of the sponge: a quadratic profile of width nb whose
// round-trip amplitude decay at normal incidence is 10^-3, exp(-2 int eta dx
// / v) = 10^-3 with int_0^{nb dx} eta_max (x / (nb dx))^2 dx = eta_max nb dx / 3,
// i.e. eta_max = 3 v_max ln(10^3) / (2 nb dx).
double default_eta_max(double vmax, int nb, double dx)
{
    return nb > 0 ? 3.0 * vmax * std::log(1000.0) / (2.0 * nb * dx) : 0.0;
}

struct Policy {
    int kind = FWI_CKPT_ALL;
    int every = 0;   // EVERY / ALL: segment length K
    int R = 2;       // forward ring length
    int nsnap = 0;   // snapshot slots per shot
    int ctop = 0;    // EVERY / ALL: base of the segment kept in the ring
};

bool multi_2d(const Geometry &g, int njobs);

int make_policy(const fwi_problem *p, const Geometry &g, int mode, const fwi_ckpt *ck, Policy *po)
{
    *po = Policy{};
    if (mode == FWI_MODE_FORWARD) {
        po->R = multi_2d(g, p->nshots) ? multi2d_steps() + 2 : 2;
        return FWI_OK;
    }
    if (!ck) return fail(FWI_EINVAL, "checkpoint policy is NULL");
    if (ck->reserved != 0) return fail(FWI_EINVAL, "fwi_ckpt.reserved must be 0");
    const int nt = p->nt;
    po->kind = ck->kind;
    switch (ck->kind) {
    case FWI_CKPT_ALL:
    case FWI_CKPT_EVERY: {
        int K = ck->kind == FWI_CKPT_ALL ? nt : ck->every;
        if (K < 1) return fail(FWI_EINVAL, "every must be >= 1");
        K = std::min(K, nt);
        po->every = K;
        po->R = K + 1;
        po->ctop = K * ((nt - 1) / K);
        po->nsnap = std::max(0, po->ctop / K - 1);
        return FWI_OK;
    }
    case FWI_CKPT_REVOLVE: {
        po->R = 2;
        if (ck->slots < 0) return fail(FWI_EINVAL, "slots must be >= 0");
        if (ck->slots > 0) {
            po->nsnap = ck->slots;
        } else {
            const uint64_t per = 2ull * (uint64_t)g.fstride * sizeof(float) * (uint64_t)p->nshots;
            po->nsnap = (int)std::min<uint64_t>(ck->budget_bytes / per, (uint64_t)nt);
        }
        po->nsnap = std::min(po->nsnap, nt);
        return FWI_OK;
    }
    default:
        return fail(FWI_EINVAL, "unknown checkpoint kind %d", ck->kind);
    }
}

// Upper bound on the tiles of one 2-D adjoint launch per shot (chunks are at
// least one row): sizes the per-tile receiver lists before the tiling is
// chosen.
uint64_t max_adj_tiles_2d(const Geometry &g)
{
    return (uint64_t)((g.nx + g.M + kTileX - 1) / kTileX) * (uint64_t)g.nz;
}

// Byte layout of the workspace (ws) and of the checkpoint buffer (ck).
struct Layout {
    uint64_t kappa = 0, ring = 0, adj = 0, grad = 0, snap = 0;
    uint64_t jobs = 0, prefix = 0, rec_off = 0, rec_next = 0, rec_head = 0, rt_start = 0, rt_rec = 0;
    uint64_t rt_key = 0;
    uint64_t res = 0, partial = 0, misfit = 0, fold1 = 0, fold2 = 0, vstats = 0;
    bool ring_in_ws = false, has_adj = false, has_res = false, has_fold = false;
    uint64_t ws_total = 0, ck_total = 0;
};

struct Carver {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes)
    {
        const uint64_t o = off;
        off = align_up(off + bytes, kAlign);
        return o;
    }
};

void make_layout(const fwi_problem *p, const Geometry &g, const Policy &po, int mode, Layout *L)
{
    *L = Layout{};
    const uint64_t S = (uint64_t)p->nshots, R = (uint64_t)p->nrec;
    const uint64_t fb = (uint64_t)g.fstride * sizeof(float);
    const int njobs = p->nshots;
    Carver w;
    L->kappa = w.take(fb);
    L->jobs = w.take(sizeof(Job) * (uint64_t)njobs);
    L->prefix = w.take(sizeof(int) * 3ull * (njobs + 1));
    L->rec_off = w.take(sizeof(int64_t) * S * R + 8);
    L->rec_next = w.take(sizeof(int32_t) * S * R + 4);
    L->rec_head = w.take(sizeof(int32_t) * S * R + 4);
    if (g.ndim == 2) {
        L->rt_start = w.take(sizeof(int32_t) * S * (max_adj_tiles_2d(g) + 1));
        L->rt_rec = w.take(sizeof(int32_t) * S * R + 4);
        L->rt_key = w.take(sizeof(int32_t) * S * R + 4);
    }
    L->vstats = w.take(sizeof(float) * 3ull * vstats_blocks());
    if (mode == FWI_MODE_BACKWARD || mode == FWI_MODE_GRADIENT) {
        L->has_adj = true;
        L->adj = w.take(2 * fb * S);
        L->grad = w.take(fb * S);
        L->has_fold = true;
        L->fold1 = w.take(sizeof(float) * (uint64_t)g.nz * g.ny * g.nxm);
        L->fold2 = w.take(sizeof(float) * (uint64_t)g.nz * g.nym * g.nxm);
    }
    if (mode == FWI_MODE_GRADIENT) {
        L->has_res = true;
        L->res = w.take(sizeof(float) * S * (uint64_t)p->nt * R + 4);
        L->partial = w.take(sizeof(double) * (uint64_t)misfit_partials());
        L->misfit = w.take(sizeof(double));
    }
    // wavefield ring and snapshots
    Carver c;
    const uint64_t ring = c.take(fb * S * (uint64_t)po.R);
    const uint64_t snap = c.take(2 * fb * S * (uint64_t)po.nsnap);
    if (mode == FWI_MODE_FORWARD || mode == FWI_MODE_GRADIENT) {
        L->ring_in_ws = true;
        const uint64_t base = w.take(c.off);
        L->ring = base + ring;
        L->snap = base + snap;
    } else {
        L->ring = ring;
        L->snap = snap;
    }
    L->ws_total = w.off;
    L->ck_total = c.off;
}

// 3-D block shape code: 4 (4 wavefronts, 4 rows per thread), 8 (8, 4),
// 42 (4 wavefronts, 2 rows per thread) or 82 (8, 2).  8th-order forward
// launches default to 4 (188 registers, 2 waves per SIMD, 85 us per step on
// a 304^3 grid; 82: 90 us, 42: 93 us).  The adjoint, which carries two
// fields, and the 16th-order stencil, which needs twice the queue, default
// to 42 (3 waves per SIMD; on the same grid the 8th-order fused adjoint
// makes the 600-step gradient 0.207 s against 0.215 s with 82, the
// 16th-order forward takes 101 against 129 us: 8-wave blocks of 3 waves per
// SIMD leave one block per CU).
int shape_code(bool adj, int M)
{
    if (const char *e = getenv(adj ? "FWI_WAVES_ADJ" : "FWI_WAVES")) {
        const int v = atoi(e);
        if (v == 4 || v == 8 || v == 42 || v == 82) return v;
    }
    return adj || M >= 8 ? 42 : 4;
}
// 2-D launches: grids too small to fill the GPU take the one-cell-per-lane
// kernel with one-row tiles (shape code 1), whose launch is one round of load
// latency; larger ones the marching kernel (code 4), which reads each field
// once.  The split is by the cells one launch updates (FWI_DIRECT2D=0/1
// forces either).
constexpr int64_t kDirect2dCells = 1 << 21;
bool direct_2d(const Geometry &g, int njobs)
{
    if (g.ndim != 2) return false;
    if (const char *e = getenv("FWI_DIRECT2D")) return atoi(e) != 0;
    return (int64_t)njobs * g.nz * g.nx <= kDirect2dCells;
}
// Forward-only calls on such grids (up to 8th order) advance several steps
// per launch (k_step2d_multi); their ring holds K + 2 levels so that a
// launch's input slots (n, n-1) and output slots (n+kk, n+kk-1) differ.
// FWI_MULTI2D=0 keeps one step per launch.
bool multi_2d(const Geometry &g, int njobs)
{
    if (g.ndim != 2 || g.M > 4 || !direct_2d(g, njobs)) return false;
    const char *e = getenv("FWI_MULTI2D");
    return !e || atoi(e) != 0;
}

int block_waves(int code) { return code == 8 || code == 82 ? 8 : 4; }
int block_rows(int code) { return code == 42 || code == 82 ? 2 : 4; }

void tiles_for(const Geometry &g, int njobs, bool adj, int *ntx, int *nty, int *nzc, int *zc)
{
    const int M = g.M;
    const int code = shape_code(adj, g.M);
    const int ty = block_rows(code) * block_waves(code);
    *ntx = (g.nx + M + kTileX - 1) / kTileX;
    *nty = g.ndim == 3 ? (g.ny + ty - 1) / ty : 1;
    const int64_t per = (int64_t)(*ntx) * (*nty) * njobs;
    int z;
    if (g.ndim == 3) {
        // 3-D: the chunk count is chosen by how well the blocks fill whole
        // waves of resident blocks (occupancy x CUs: a partial last wave idles
        // part of the GPU) against the cost of short chunks (each warms its
        // z-queue with 2M extra planes of the stencil field before its first
        // plane).  Scored as (1 + M / zc) x (w + 7/8 (ceil(w) - w)) / w for w
        // waves: the warm-up weighs twice its share of the bytes (it is also
        // serial latency), and a partial last wave costs 7/8 of a full one
        // (its blocks share the bandwidth among fewer).  The weights fit the
        // measured chunk sweeps at 2 blocks per CU: 304^3 padded, 8th order:
        // 5 chunks of 61 planes (475 blocks, 84.7 us; 38 planes 101 us, 76
        // planes 95 us); 560 x 560 x 304: 3 chunks of 102 (forward 1.4 %
        // faster than 8 of 38); a 128 x 1024 x 1024 slab: 4 chunks of 32
        // (477 against 502 us with 6 of 22).  Chunks are at least 4 planes.
        static int cus = 0;
        if (cus == 0) {
            int dev = 0;
            hipDeviceProp_t prop;
            if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
                cus = prop.multiProcessorCount;
            if (cus <= 0) cus = 256;
        }
        const int occ = std::max(1, step_blocks_per_cu(3, g.M, code, adj));
        int64_t slots = (int64_t)occ * cus;
        if (const char *e = getenv("FWI_TARGET_BLOCKS")) slots = std::max(1, atoi(e));
        double best = 0.0;
        z = g.nz;
        for (int n = 1; n <= std::max(1, g.nz / 4); ++n) {
            const int zc = (g.nz + n - 1) / n;
            const int nc = (g.nz + zc - 1) / zc;
            const double waves = (double)(per * nc) / (double)slots;
            const double tail = (waves + 0.875 * (std::ceil(waves) - waves)) / waves;
            const double score = (1.0 + (double)M / zc) * tail;
            if (n == 1 || score < best - 1e-12) {
                best = score;
                z = zc;
            }
        }
    } else if (direct_2d(g, njobs)) {
        *zc = 1;   // one-row tiles of the one-cell-per-lane kernel
        *nzc = g.nz;
        return;
    } else {
        // 2-D fields are small and largely cache-resident: many short chunks
        // (16384 blocks: 12-row chunks for 32 shots of 1064 x 360, 8 % faster
        // than 8192 on the 2-D gradient)
        int64_t target = 16384;
        if (const char *e = getenv("FWI_TARGET_BLOCKS")) target = std::max(1, atoi(e));
        const int want = (int)std::max<int64_t>(1, (target + per - 1) / per);
        z = (g.nz + want - 1) / want;
    }
    // at least 4 planes per chunk: grids too small to fill the GPU are bound
    // by the serial plane loop of each block, and 4-plane chunks beat 8-plane
    // ones there (one 1064 x 360 2-D shot: +29 %)
    z = std::max(z, std::min(g.nz, 4));
    if (const char *e = getenv("FWI_ZCHUNK")) z = std::max(1, atoi(e));
    z = std::min(z, g.nz);
    *zc = z;
    *nzc = (g.nz + z - 1) / z;
}

// z-chunk order and marching direction of 3-D step launches (kTile* flags).
int tile_flags(const Geometry &g)
{
    if (g.ndim != 3) return 0;
    int f = 0;
    if (const char *e = getenv("FWI_ZFAST")) f |= atoi(e) ? kTileZFast : 0;
    if (const char *e = getenv("FWI_ZALT")) f |= atoi(e) ? kTileZAlt : 0;
    return f;
}

int gather_threads(const Geometry &g)
{
    return g.ndim == 3 ? 64 * block_waves(shape_code(false, g.M)) : 64;
}

// ------------------------------------------------------------ call context
struct Ctx {
    const fwi_problem *p = nullptr;
    Geometry g;
    Policy po;
    Layout L;
    hipStream_t st = nullptr;
    char *ws = nullptr;
    char *ck = nullptr;
    std::vector<Job> jobs;
    Job *d_jobs = nullptr;
    int *d_prefix = nullptr;
    int ttiles = 0, atiles = 0, gblocks = 0, gthreads = 64;
    int remap = 1;
    int nw = 4, nw_adj = 42;
    // forward-only small 2-D calls: several steps per launch over
    // mtiles = mntx x (rows of tiles) output tiles per shot
    bool multi = false;
    int mtiles = 0, mntx = 0;
    std::vector<int> slot_time;
    // plan mode (host only): launches are recorded here instead of issued,
    // ten int32 per launch (see fwi_revolve_plan)
    std::vector<int32_t> *plan = nullptr;

    float *f_at(uint64_t off, bool in_ws) const
    {
        return reinterpret_cast<float *>((in_ws ? ws : ck) + off);
    }
};

int prepare(Ctx &c, const fwi_problem *p, int mode, const fwi_ckpt *ck, void *ws,
            uint64_t ws_bytes, void *ckbuf, uint64_t ck_bytes, void *stream)
{
    int st = make_geometry(p, &c.g);
    if (st) return st;
    c.p = p;
    st = make_policy(p, c.g, mode, ck, &c.po);
    if (st) return st;
    make_layout(p, c.g, c.po, mode, &c.L);
    if (!ws) return fail(FWI_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0)
        return fail(FWI_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < c.L.ws_total)
        return fail(FWI_ENOMEM, "workspace too small: %llu < %llu bytes",
                    (unsigned long long)ws_bytes, (unsigned long long)c.L.ws_total);
    if (!c.L.ring_in_ws) {
        if (!ckbuf) return fail(FWI_EINVAL, "checkpoint buffer is NULL");
        if ((reinterpret_cast<uintptr_t>(ckbuf) & (kAlign - 1)) != 0)
            return fail(FWI_EINVAL, "checkpoint buffer must be 256-byte aligned");
        if (ck_bytes < c.L.ck_total)
            return fail(FWI_ENOMEM, "checkpoint buffer too small: %llu < %llu bytes",
                        (unsigned long long)ck_bytes, (unsigned long long)c.L.ck_total);
    }
    c.ws = static_cast<char *>(ws);
    c.ck = static_cast<char *>(ckbuf);
    c.st = static_cast<hipStream_t>(stream);
    if (const char *e = getenv("FWI_XCD_REMAP")) c.remap = atoi(e) != 0;
    c.nw = shape_code(false, c.g.M);
    c.nw_adj = shape_code(true, c.g.M);
    if (c.g.ndim == 2) c.nw = c.nw_adj = direct_2d(c.g, p->nshots) ? 1 : 4;
    c.multi = mode == FWI_MODE_FORWARD && multi_2d(c.g, p->nshots) &&
              c.po.R == multi2d_steps() + 2;
    if (c.multi) {
        int ox = 0, oz = 0;
        multi2d_tile(c.g.M, &ox, &oz);
        c.mntx = (c.g.nx + ox - 1) / ox;
        c.mtiles = c.mntx * ((c.g.nz + oz - 1) / oz);
    }
    return FWI_OK;
}

// Reads positions and model statistics back, checks them, and uploads the
// job table.  res: adjoint source (or NULL); traces: recording target (or NULL).
int stage(Ctx &c, const float *v, const float *src, const int32_t *src_pos,
          const int32_t *rec_pos, float *traces, const float *res, int accumulate)
{
    const fwi_problem *p = c.p;
    const Geometry &g = c.g;
    const int S = p->nshots, R = p->nrec, D = p->ndim;
    if (!v || !src_pos || (R > 0 && !rec_pos)) return fail(FWI_EINVAL, "NULL input array");
    std::vector<int32_t> hs((size_t)S * D), hr((size_t)S * R * D);
    HIP_TRY(hipMemcpyAsync(hs.data(), src_pos, hs.size() * 4, hipMemcpyDeviceToHost, c.st));
    if (!hr.empty())
        HIP_TRY(hipMemcpyAsync(hr.data(), rec_pos, hr.size() * 4, hipMemcpyDeviceToHost, c.st));
    float *d_vs = c.f_at(c.L.vstats, true);
    launch_vstats(v, g.model_cells, d_vs, c.st);
    HIP_TRY(hipGetLastError());
    std::vector<float> hv(3 * (size_t)vstats_blocks());
    HIP_TRY(hipMemcpyAsync(hv.data(), d_vs, hv.size() * 4, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));

    const int dims[3] = {g.nzm, g.nym, g.nxm};
    auto in_model = [&](const int32_t *q) {
        if (D == 2) return q[0] >= 0 && q[0] < dims[0] && q[1] >= 0 && q[1] < dims[2];
        return q[0] >= 0 && q[0] < dims[0] && q[1] >= 0 && q[1] < dims[1] && q[2] >= 0 &&
               q[2] < dims[2];
    };
    for (int s = 0; s < S; ++s)
        if (!in_model(&hs[(size_t)s * D])) return fail(FWI_EBOUNDS, "source %d outside the model", s);
    for (size_t r = 0; r < (size_t)S * R; ++r)
        if (!in_model(&hr[r * D])) return fail(FWI_EBOUNDS, "receiver %zu outside the model", r);

    const int B = vstats_blocks();
    float vmin = INFINITY, vmax = -INFINITY, bad = 0.f;
    for (int i = 0; i < B; ++i) {
        vmin = std::min(vmin, hv[i]);
        vmax = std::max(vmax, hv[B + i]);
        bad += hv[2 * B + i];
    }
    if (bad > 0.f) return fail(FWI_EINVAL, "velocity has non-finite values");
    if (!(vmin > 0.f)) return fail(FWI_EINVAL, "velocity must be > 0 (min %g)", (double)vmin);
    const double cfl = (double)vmax * p->dt / p->dx;
    const double lim = std::sqrt(4.0 / (p->ndim * max_symbol(p->order)));
    if (cfl > lim) return fail(FWI_ECFL, "v_max dt / dx = %.4f exceeds %.4f", cfl, lim);
    // sponge strength: as given, or (eta_max < 0) the default for this model
    const double eta_max = p->eta_max >= 0.f ? (double)p->eta_max
                                             : default_eta_max(vmax, g.nb, p->dx);

    // receiver offsets and duplicate chains (receivers sharing a cell)
    auto offset = [&](const int32_t *q) -> int64_t {
        const int z = q[0] + g.nb;
        const int y = D == 3 ? q[1] + g.nb : 0;
        const int x = (D == 3 ? q[2] : q[1]) + g.nb;
        return ((int64_t)(z + g.M) * g.nya + (y + g.gy)) * g.pitch + (x + g.M);
    };
    std::vector<int64_t> roff((size_t)S * R);
    std::vector<int32_t> rnext((size_t)S * R, -1), rhead((size_t)S * R, 0);
    std::vector<int32_t> order(R);
    for (int s = 0; s < S; ++s) {
        int64_t *o = roff.data() + (size_t)s * R;
        for (int r = 0; r < R; ++r) o[r] = offset(&hr[((size_t)s * R + r) * D]);
        for (int r = 0; r < R; ++r) order[r] = r;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return o[a] < o[b]; });
        for (int i = 0; i < R; ++i) {
            const int r = order[i];
            const bool first = i == 0 || o[order[i - 1]] != o[r];
            rhead[(size_t)s * R + r] = first ? 1 : 0;
            if (i + 1 < R && o[order[i + 1]] == o[r]) rnext[(size_t)s * R + r] = order[i + 1];
        }
    }

    // job table: one job per shot
    Job::Tiling til[2];
    for (int a = 0; a < 2; ++a) {
        tiles_for(g, S, a == 1, &til[a].ntx, &til[a].nty, &til[a].nzc, &til[a].zc);
        til[a].ntiles = til[a].ntx * til[a].nty * til[a].nzc;
        til[a].flags = tile_flags(g);
    }
    c.gthreads = gather_threads(g);
    const int ng = (R + c.gthreads - 1) / c.gthreads;
    const uint64_t fs = (uint64_t)g.fstride;
    float *kappa = c.f_at(c.L.kappa, true);
    float *ring = c.f_at(c.L.ring, c.L.ring_in_ws);
    float *snap = c.f_at(c.L.snap, c.L.ring_in_ws);
    float *adj = c.L.has_adj ? c.f_at(c.L.adj, true) : nullptr;
    float *grad = c.L.has_adj ? c.f_at(c.L.grad, true) : nullptr;
    int64_t *d_roff = reinterpret_cast<int64_t *>(c.ws + c.L.rec_off);
    int32_t *d_rnext = reinterpret_cast<int32_t *>(c.ws + c.L.rec_next);
    int32_t *d_rhead = reinterpret_cast<int32_t *>(c.ws + c.L.rec_head);
    // 2-D adjoint source lists: each receiver cell (its first receiver) under
    // the adjoint tile that stores it, sorted by tile and then by row
    const bool lists = D == 2;
    const uint64_t mt = lists ? max_adj_tiles_2d(g) + 1 : 0;
    int32_t *d_rtstart = lists ? reinterpret_cast<int32_t *>(c.ws + c.L.rt_start) : nullptr;
    int32_t *d_rtrec = lists ? reinterpret_cast<int32_t *>(c.ws + c.L.rt_rec) : nullptr;
    int32_t *d_rtkey = lists ? reinterpret_cast<int32_t *>(c.ws + c.L.rt_key) : nullptr;
    std::vector<int32_t> rtstart((size_t)S * mt, 0), rtrec(lists ? (size_t)S * R : 0);
    std::vector<int32_t> rtkey(rtrec.size());
    if (lists) {
        const Job::Tiling &T = til[1];
        std::vector<std::pair<int64_t, int32_t>> key;
        for (int s = 0; s < S; ++s) {
            key.clear();
            for (int r = 0; r < R; ++r) {
                if (!rhead[(size_t)s * R + r]) continue;
                const int64_t off = roff[(size_t)s * R + r];
                const int zr = (int)(off / g.pitch) - g.M, cr = (int)(off % g.pitch);
                const int64_t tile = (int64_t)(zr / T.zc) * T.ntx + cr / kTileX;
                key.push_back({(tile * (int64_t)(g.nz + 1) + zr) * kTileX + cr % kTileX, r});
            }
            std::stable_sort(key.begin(), key.end());
            int32_t *st = &rtstart[(size_t)s * mt];
            int32_t *lst = &rtrec[(size_t)s * R];
            int32_t *kk = &rtkey[(size_t)s * R];
            for (size_t i = 0; i < key.size(); ++i) {
                const int64_t tz = key[i].first / kTileX;   // tile * (nz + 1) + row
                lst[i] = key[i].second;
                kk[i] = (int32_t)((tz % (g.nz + 1)) << 6 | (key[i].first % kTileX));
                st[tz / (g.nz + 1) + 1] += 1;
            }
            for (uint64_t t = 1; t < mt; ++t) st[t] += st[t - 1];
        }
    }
    double cell = 1.0;
    for (int a = 0; a < D; ++a) cell *= p->dx;
    c.jobs.assign(S, Job{});
    // [forward tile prefix | gather prefix | adjoint tile prefix], S+1 each
    std::vector<int> prefix(3 * (S + 1), 0);
    for (int s = 0; s < S; ++s) {
        Job &J = c.jobs[s];
        J.nz = g.nz; J.ny = g.ny; J.nx = g.nx;
        J.pitch = g.pitch; J.nya = g.nya; J.nb = g.nb;
        J.plane = g.plane; J.fstride = g.fstride;
        J.eta_dt = g.nb > 0 ? (float)(eta_max * p->dt / ((double)g.nb * g.nb)) : 0.f;
        J.src_scale = (float)((double)p->dt * p->dt / cell);
        J.tile[0] = til[0];
        J.tile[1] = til[1];
        J.ngather = ng;
        J.n0 = 0; J.k0 = 0; J.nt = p->nt;
        J.fwd_lo = 0; J.fwd_hi = p->nt;
        J.adj_lo = 1; J.adj_hi = p->nt + 1;
        J.record = traces != nullptr;
        J.accumulate = accumulate;
        J.kappa = kappa;
        J.ring = ring + (uint64_t)s * c.po.R * fs;
        J.R = c.po.R;
        J.adj = adj ? adj + (uint64_t)s * 2 * fs : nullptr;
        J.grad = grad ? grad + (uint64_t)s * fs : nullptr;
        J.snap = c.po.nsnap > 0 ? snap + (uint64_t)s * 2 * c.po.nsnap * fs : nullptr;
        const int32_t *q = &hs[(size_t)s * D];
        J.src_z = q[0] + g.nb;
        J.src_y = D == 3 ? q[1] + g.nb : 0;
        J.src_x = (D == 3 ? q[2] : q[1]) + g.nb;
        J.nrec = R;
        J.wavelet = src ? src + (size_t)s * p->nt : nullptr;
        J.rec_off = d_roff + (size_t)s * R;
        J.rec_next = d_rnext + (size_t)s * R;
        J.rec_head = d_rhead + (size_t)s * R;
        J.rt_start = lists ? d_rtstart + (size_t)s * mt : nullptr;
        J.rt_rec = lists ? d_rtrec + (size_t)s * R : nullptr;
        J.rt_key = lists ? d_rtkey + (size_t)s * R : nullptr;
        J.traces = traces ? traces + (size_t)s * p->nt * R : nullptr;
        J.res = res ? res + (size_t)s * p->nt * R : nullptr;
        prefix[s + 1] = prefix[s] + J.tile[0].ntiles;
        prefix[S + 1 + s + 1] = prefix[S + 1 + s] + ng;
        prefix[2 * (S + 1) + s + 1] = prefix[2 * (S + 1) + s] + J.tile[1].ntiles;
    }
    c.ttiles = prefix[S];
    c.gblocks = prefix[2 * S + 1];
    c.atiles = prefix[3 * S + 2];
    c.d_jobs = reinterpret_cast<Job *>(c.ws + c.L.jobs);
    c.d_prefix = reinterpret_cast<int *>(c.ws + c.L.prefix);
    HIP_TRY(hipMemcpyAsync(c.d_jobs, c.jobs.data(), sizeof(Job) * S, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(c.d_prefix, prefix.data(), sizeof(int) * prefix.size(),
                           hipMemcpyHostToDevice, c.st));
    if (lists) {
        HIP_TRY(hipMemcpyAsync(d_rtstart, rtstart.data(), rtstart.size() * 4,
                               hipMemcpyHostToDevice, c.st));
        if (R > 0) {
            HIP_TRY(hipMemcpyAsync(d_rtrec, rtrec.data(), rtrec.size() * 4,
                                   hipMemcpyHostToDevice, c.st));
            HIP_TRY(hipMemcpyAsync(d_rtkey, rtkey.data(), rtkey.size() * 4,
                                   hipMemcpyHostToDevice, c.st));
        }
    }
    if (R > 0) {
        HIP_TRY(hipMemcpyAsync(d_roff, roff.data(), roff.size() * 8, hipMemcpyHostToDevice, c.st));
        HIP_TRY(hipMemcpyAsync(d_rnext, rnext.data(), rnext.size() * 4, hipMemcpyHostToDevice, c.st));
        HIP_TRY(hipMemcpyAsync(d_rhead, rhead.data(), rhead.size() * 4, hipMemcpyHostToDevice, c.st));
    }
    // model -> kappa' = (v dt/dx)^2 on the padded grid
    launch_prep_kappa(v, kappa, g.M, g.gy, g.nz, g.ny, g.nx, g.pitch, g.nya, g.nb, g.nzm, g.nym,
                      g.nxm, g.fstride, (float)((double)p->dt / p->dx), c.st);
    HIP_TRY(hipGetLastError());
    // host staging vectors die with this frame: finish the uploads now
    HIP_TRY(hipStreamSynchronize(c.st));
    return FWI_OK;
}

#define TRY(x)                   \
    do {                         \
        const int s_ = (x);      \
        if (s_) return s_;       \
    } while (0)

// ------------------------------------------------------------ time loops
void plan_op(Ctx &c, int kind, int a, int b, int d, const LevelMap &lm)
{
    const int32_t row[10] = {kind, a, b, d, lm.lev[0], lm.fld[0], lm.lev[1], lm.fld[1],
                             lm.lev[2], lm.fld[2]};
    c.plan->insert(c.plan->end(), row, row + 10);
}

int fwd_step(Ctx &c, int n, bool record, const LevelMap &lm = LevelMap{})
{
    if (c.plan) { plan_op(c, 1, n, 0, 0, lm); return FWI_OK; }
    launch_step(c.g.ndim, c.g.M, c.nw, false, c.d_jobs, c.d_prefix, c.p->nshots, n, c.ttiles,
                record ? c.gblocks : 0, c.remap, lm, c.st);
    return FWI_OK;
}

int adj_step(Ctx &c, int k, const LevelMap &lm = LevelMap{})
{
    if (c.plan) { plan_op(c, 2, k, 0, 0, lm); return FWI_OK; }
    launch_step(c.g.ndim, c.g.M, c.nw_adj, true, c.d_jobs, c.d_prefix + 2 * (c.p->nshots + 1),
                c.p->nshots, -k, c.atiles, 0, c.remap, lm, c.st);
    if (c.g.ndim == 3)   // 2-D adjoint steps add the adjoint source themselves
        launch_adj_inject(c.d_jobs, c.d_prefix + c.p->nshots + 1, c.p->nshots, c.gblocks,
                          c.gthreads, -k, c.st);
    return FWI_OK;
}

// dir 0: levels time, time-1 -> slot (read where lm puts them); 1: slot ->
// ring; 2: zero levels 0, -1 in the ring.  mask bit w: level time - w.
int snapshot(Ctx &c, int slot, int time, int dir, int mask = 3, const LevelMap &lm = LevelMap{})
{
    if (dir != 2 && (slot < 0 || slot >= c.po.nsnap))
        return fail(FWI_EINVAL, "internal: snapshot slot %d of %d", slot, c.po.nsnap);
    if (c.plan) { plan_op(c, 3, slot, time, dir | mask << 2, lm); return FWI_OK; }
    launch_snapshot(c.d_jobs, c.p->nshots, c.g.fstride, slot, time, dir, mask, lm, c.st);
    return FWI_OK;
}

// Binomial checkpointing without snapshot copies.  A restore does not copy
// the slot back into the ring: the following steps (or the adjoint step)
// read the two levels from the slot.  The steps that produce the two levels
// of a snapshot write them into the slot, and the steps after read them
// there.  Held lists the live forward levels kept in snapshot fields; every
// other level is in the ring.  A copy remains only where a snapshot follows
// fewer than two steps, and FWI_REVOLVE_COPY=1 restores copies throughout.
struct Held {
    std::vector<std::pair<int, int>> at;   // (level, snapshot field 2s + w)

    int field(int L) const
    {
        for (const auto &e : at)
            if (e.first == L) return e.second;
        return -1;
    }
    void put(int L, int f)
    {
        drop_if([L](const std::pair<int, int> &e) { return e.first == L; });
        if (f >= 0) at.push_back({L, f});
    }
    void keep_from(int L)
    {
        drop_if([L](const std::pair<int, int> &e) { return e.first < L; });
    }
    bool uses_slot(int slot) const
    {
        for (const auto &e : at)
            if (e.second / 2 == slot) return true;
        return false;
    }
    template <class F>
    void drop_if(F f)
    {
        at.erase(std::remove_if(at.begin(), at.end(), f), at.end());
    }
    // map entries for the listed levels that live in snapshot fields
    LevelMap map(std::initializer_list<int> levels) const
    {
        LevelMap m;
        int i = 0;
        for (int L : levels) {
            const int f = field(L);
            if (f >= 0 && i < 3) { m.lev[i] = L; m.fld[i] = f; ++i; }
        }
        return m;
    }
};

bool revolve_copies()
{
    const char *e = getenv("FWI_REVOLVE_COPY");
    return e && atoi(e) != 0;
}

// Forward step n -> n+1: levels n and n-1 read where they are held, level
// n+1 written to snapshot field dst (-1: the ring).
void rv_step(Ctx &c, Held &h, int n, bool record, int dst)
{
    LevelMap m = h.map({n, n - 1});
    if (dst >= 0) {
        int i = 0;
        while (i < 3 && m.lev[i] != kNoLevel) ++i;
        m.lev[i] = n + 1;   // i < 3: at most two entries above
        m.fld[i] = dst;
    }
    fwd_step(c, n, record, m);
    h.put(n + 1, dst);
    h.keep_from(n);
}

// Advance cur -> to.  If a snapshot into slot `shot` (-1: none) follows at
// time `to`, the steps producing levels to - 1 and to write into the slot,
// unless a live level is held there.
void rv_advance(Ctx &c, Held &h, int cur, int to, int shot, bool record)
{
    const bool direct = shot >= 0 && !revolve_copies() && !h.uses_slot(shot);
    for (int n = cur; n < to; ++n) {
        int dst = -1;
        if (direct && n + 1 == to) dst = 2 * shot;
        else if (direct && n + 1 == to - 1) dst = 2 * shot + 1;
        rv_step(c, h, n, record, dst);
    }
}

// Snapshot of levels t, t-1 into slot: copies what the steps did not write
// there.  A source held in the other field of the same slot is copied first,
// in a launch of its own.  (The binomial schedules never do this: a slot is
// not overwritten one step after it was restored.)
int rv_takeshot(Ctx &c, Held &h, int slot, int t)
{
    const int mask = (h.field(t) != 2 * slot ? 1 : 0) | (h.field(t - 1) != 2 * slot + 1 ? 2 : 0);
    const LevelMap m = h.map({t, t - 1});
    if (mask == 3 && h.field(t - 1) == 2 * slot) {
        TRY(snapshot(c, slot, t, 0, 2, m));
        TRY(snapshot(c, slot, t, 0, 1, m));
    } else if (mask == 3 && h.field(t) == 2 * slot + 1) {
        TRY(snapshot(c, slot, t, 0, 1, m));
        TRY(snapshot(c, slot, t, 0, 2, m));
    } else if (mask) {
        TRY(snapshot(c, slot, t, 0, mask, m));
    }
    return FWI_OK;
}

// Restore of slot (time t): the levels stay in the slot.
int rv_restore(Ctx &c, Held &h, int slot, int t)
{
    h.at.clear();
    if (revolve_copies()) return snapshot(c, slot, t, 1);
    h.put(t, 2 * slot);
    h.put(t - 1, 2 * slot + 1);
    return FWI_OK;
}

// Copies held levels back into the ring (field f holds level L).
int rv_to_ring(Ctx &c, Held &h, int L)
{
    const int f = h.field(L);
    if (f < 0) return FWI_OK;
    TRY(snapshot(c, f / 2, L + (f & 1), 1, 1 << (f & 1)));
    h.put(L, -1);
    return FWI_OK;
}


void zero(float *p, uint64_t floats, hipStream_t st) { launch_fill(p, (int64_t)floats, 0.f, st); }

// Frames and row padding of nf consecutive fields.  Step kernels never store
// there and read it as the zero boundary; grid cells of a level are all
// written by the step that produces it before anything reads them, so a
// level store needs only its frames cleared (and the initial levels 0 and -1
// cleared whole).  For a checkpoint ring kept whole in HBM this is ~10 % of
// the bytes of a full clear.
void zero_frames(const Ctx &c, float *p, uint64_t nf)
{
    const Geometry &g = c.g;
    launch_zero_frames(p, (int64_t)nf, g.fstride, g.nya, g.pitch, g.M, g.gy, g.nz, g.ny, g.nx,
                       c.st);
}

// Forward sweep 0 -> nt recording traces and taking the policy's snapshots.
int forward_phase(Ctx &c, bool record)
{
    const int nt = c.p->nt;
    const uint64_t fs = (uint64_t)c.g.fstride;
    if (!c.plan) {
        zero_frames(c, c.jobs[0].ring, (uint64_t)c.po.R * c.p->nshots);
        TRY(snapshot(c, 0, 0, 2));   // levels 0 and -1: the zero initial state
    }
    if (c.po.kind == FWI_CKPT_REVOLVE) {
        int64_t steps = 0;
        std::vector<Action> acts = revolve_schedule(nt, c.po.nsnap, &steps);
        c.slot_time.assign(std::max(c.po.nsnap, 1), -1);
        // steps store only grid cells, so fields they write must start with
        // a zero frame: the snapshot store is cleared once
        if (!revolve_copies() && c.po.nsnap > 0 && !c.plan)
            zero_frames(c, c.jobs[0].snap, 2 * (uint64_t)c.po.nsnap * c.p->nshots);
        int cur = 0;
        Held h;
        for (size_t i = 0; i < acts.size() && acts[i].op != OP_ADJOINT; ++i) {
            const Action &a = acts[i];
            if (a.op == OP_ADVANCE) {
                const bool shot = i + 1 < acts.size() && acts[i + 1].op == OP_TAKESHOT;
                rv_advance(c, h, cur, a.arg, shot ? acts[i + 1].arg : -1, record);
                cur = a.arg;
            } else if (a.op == OP_TAKESHOT) {
                TRY(rv_takeshot(c, h, a.arg, cur));
                c.slot_time[a.arg] = cur;
            } else {
                return fail(FWI_EINVAL, "revolve: unexpected action in the first sweep");
            }
        }
        for (int n = cur; n < nt; ++n) rv_step(c, h, n, record, -1);
        // the end state goes to the ring, where the backward sweep (possibly a
        // separate call) starts
        if (record)
            launch_gather(c.d_jobs, c.d_prefix + c.p->nshots + 1, c.p->nshots, c.gblocks,
                          c.gthreads, nt, h.map({nt}), c.st);
        TRY(rv_to_ring(c, h, nt));
        TRY(rv_to_ring(c, h, nt - 1));
        if (!c.plan) HIP_TRY(hipGetLastError());
        return FWI_OK;
    } else if (c.multi && !c.plan) {
        // up to multi2d_steps() steps per launch; a last single step runs alone
        for (int n = 0; n < nt;) {
            const int kk = std::min(nt - n, multi2d_steps());
            if (kk >= 2) {
                launch_step2d_multi(c.g.M, c.d_jobs, c.p->nshots, c.mtiles, c.mntx, n, kk, record,
                                    c.st);
            } else {
                fwd_step(c, n, record);
            }
            n += kk;
        }
    } else {
        const int K = c.po.every;
        for (int n = 0; n < nt; ++n) {
            fwd_step(c, n, record);
            const int t = n + 1;
            if (K > 0 && t % K == 0 && t <= c.po.ctop - K) TRY(snapshot(c, t / K - 1, t, 0));
        }
    }
    if (record)
        launch_gather(c.d_jobs, c.d_prefix + c.p->nshots + 1, c.p->nshots, c.gblocks,
                      c.gthreads, nt, LevelMap{}, c.st);
    HIP_TRY(hipGetLastError());
    return FWI_OK;
}

// Adjoint sweep k = nt .. 1 with gradient accumulation; assumes the ring
// holds the end state of forward_phase.
int backward_phase(Ctx &c)
{
    const int nt = c.p->nt;
    const uint64_t fs = (uint64_t)c.g.fstride;
    if (!c.plan) {
        zero(c.jobs[0].adj, 2 * fs * c.p->nshots, c.st);
        zero(c.jobs[0].grad, fs * c.p->nshots, c.st);
    }
    adj_step(c, nt);
    if (c.po.kind == FWI_CKPT_REVOLVE) {
        int64_t steps = 0;
        std::vector<Action> acts = revolve_schedule(nt, c.po.nsnap, &steps);
        c.slot_time.assign(std::max(c.po.nsnap, 1), -1);
        size_t i = 0;
        int cur = 0;
        for (; i < acts.size() && acts[i].op != OP_ADJOINT; ++i) {
            if (acts[i].op == OP_ADVANCE) cur = acts[i].arg;
            else if (acts[i].op == OP_TAKESHOT) c.slot_time[acts[i].arg] = cur;
        }
        cur = nt;
        Held h;   // the forward sweep left levels nt and nt-1 in the ring
        for (; i < acts.size(); ++i) {
            const Action &a = acts[i];
            switch (a.op) {
            case OP_ADJOINT: adj_step(c, a.arg, h.map({a.arg})); break;
            case OP_ADVANCE: {
                const bool shot = i + 1 < acts.size() && acts[i + 1].op == OP_TAKESHOT;
                rv_advance(c, h, cur, a.arg, shot ? acts[i + 1].arg : -1, false);
                cur = a.arg;
                break;
            }
            case OP_TAKESHOT:
                TRY(rv_takeshot(c, h, a.arg, cur));
                c.slot_time[a.arg] = cur;
                break;
            case OP_RESTORE:
                if (a.arg < 0 || a.arg >= (int)c.slot_time.size() || c.slot_time[a.arg] < 0)
                    return fail(FWI_EINVAL, "internal: restore of an empty slot");
                cur = c.slot_time[a.arg];
                TRY(rv_restore(c, h, a.arg, cur));
                break;
            case OP_RESTART: TRY(snapshot(c, 0, 0, 2)); h.at.clear(); cur = 0; break;
            default: return fail(FWI_EINVAL, "revolve: bad action");
            }
        }
    } else {
        const int K = c.po.every, ctop = c.po.ctop;
        for (int k = nt - 1; k >= std::max(ctop, 1); --k) adj_step(c, k);
        for (int base = ctop - K; base >= 0; base -= K) {
            if (base == 0) TRY(snapshot(c, 0, 0, 2));
            else TRY(snapshot(c, base / K - 1, base, 1));
            for (int n = base; n < base + K - 1; ++n) fwd_step(c, n, false);
            for (int k = base + K - 1; k >= std::max(base, 1); --k) adj_step(c, k);
        }
    }
    if (!c.plan) HIP_TRY(hipGetLastError());
    return FWI_OK;
}

// Wavefield watchdog: FWI_ENONFINITE if forward level L (in the ring) of any
// shot holds a non-finite value.  Synchronises the stream.  An unstable or
// NaN-fed propagation ends with a non-finite field, so one check of the last
// level covers the whole run at the cost of one read of it.
int check_level(Ctx &c, int L)
{
    float *d = c.f_at(c.L.vstats, true);
    launch_nonfinite_level(c.d_jobs, c.p->nshots, L, d, c.st);
    HIP_TRY(hipGetLastError());
    std::vector<float> h((size_t)vstats_blocks());
    HIP_TRY(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    float bad = 0.f;
    for (float x : h) bad += x;
    if (bad > 0.f) return fail(FWI_ENONFINITE, "the wavefield at step %d is not finite", L);
    return FWI_OK;
}

// FWI_ENONFINITE if a model-grid output (dv) holds a non-finite value.
// Synchronises the stream.
int check_model(Ctx &c, const float *a)
{
    float *d = c.f_at(c.L.vstats, true);
    launch_vstats(a, c.g.model_cells, d, c.st);
    HIP_TRY(hipGetLastError());
    const int B = vstats_blocks();
    std::vector<float> h(3 * (size_t)B);
    HIP_TRY(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
    float bad = 0.f;
    for (int i = 0; i < B; ++i) bad += h[2 * B + i];
    if (bad > 0.f) return fail(FWI_ENONFINITE, "the gradient is not finite");
    return FWI_OK;
}

int fold(Ctx &c, const float *v, float *dv)
{
    const Geometry &g = c.g;
    launch_fold(g.ndim, c.d_jobs, c.p->nshots, g.M, g.gy, g.nz, g.ny, g.nx, g.nb, g.nzm, g.nym,
                g.nxm, c.f_at(c.L.fold1, true), c.f_at(c.L.fold2, true), v, dv, c.st);
    HIP_TRY(hipGetLastError());
    return FWI_OK;
}


// ------------------------------------------------------------ serving jobs
// A job is one shot (forward or gradient) with its own device memory and a
// program of operations.  Step operations (forward or adjoint ranges) are
// executed a chunk at a time by fwi_jobs_advance, which puts the steps of all
// active jobs into shared launches; the other operations (snapshots,
// residual, fold) are per-job launches between chunks.
enum JobOpType { JOP_FWD, JOP_ADJ, JOP_SNAP, JOP_RESTORE, JOP_ZERO_STATE, JOP_GATHER,
                 JOP_MISFIT, JOP_ZERO_ADJ, JOP_FOLD };

struct JobOp {
    int type;
    int a, b;     // FWD: levels n in [a, b) are advanced; ADJ: k = a down to b
    int slot;     // SNAP / RESTORE: snapshot slot (time in a)
    int record;   // FWD: record traces
};

}  // namespace

struct fwi_job {
    fwi_problem prob;
    Ctx c;
    int kind = 0;
    int chunk = 0;
    // binomial checkpointing: the job changes direction within a chunk, so
    // its steps carry per-round levels (Job::lev) instead of one window
    bool rounds = false;
    std::vector<JobOp> ops;
    size_t head = 0;
    const float *v = nullptr, *obs = nullptr;
    float *rec = nullptr, *res = nullptr, *dv = nullptr;
    double *d_misfit = nullptr;
};

namespace {

bool is_step(const JobOp &o) { return o.type == JOP_FWD || o.type == JOP_ADJ; }

int run_immediate(fwi_job *J, const JobOp &o)
{
    Ctx &c = J->c;
    const uint64_t fs = (uint64_t)c.g.fstride;
    switch (o.type) {
    case JOP_SNAP: return snapshot(c, o.slot, o.a, 0);
    case JOP_RESTORE: return snapshot(c, o.slot, o.a, 1);
    case JOP_ZERO_STATE: return snapshot(c, 0, 0, 2);
    case JOP_GATHER:
        launch_gather(c.d_jobs, c.d_prefix + 2, 1, c.gblocks, c.gthreads, o.a, LevelMap{}, c.st);
        return FWI_OK;
    case JOP_MISFIT: {
        const int64_t n = (int64_t)J->prob.nt * J->prob.nrec;
        if (n > 0)
            launch_misfit(J->rec, J->obs, J->res, n,
                          reinterpret_cast<double *>(c.ws + c.L.partial), J->d_misfit, c.st);
        else
            launch_fill(reinterpret_cast<float *>(J->d_misfit), 4, 0.f, c.st);
        return FWI_OK;
    }
    case JOP_ZERO_ADJ:
        zero(c.jobs[0].adj, 2 * fs, c.st);
        zero(c.jobs[0].grad, fs, c.st);
        return FWI_OK;
    case JOP_FOLD: return fold(c, J->v, J->dv);
    default: return fail(FWI_EINVAL, "internal: bad job op");
    }
}

int run_immediates(fwi_job *J)
{
    while (J->head < J->ops.size() && !is_step(J->ops[J->head])) {
        TRY(run_immediate(J, J->ops[J->head]));
        ++J->head;
    }
    return FWI_OK;
}

// Revolve program, with copies: snapshots copy two levels out of the two-level
// ring and restores copy them back (the launch-wide level maps of the
// lockstep path do not apply to jobs that share launches).  The order of
// operations is that of forward_phase / backward_phase.
void build_revolve_program(fwi_job *J)
{
    const int nt = J->prob.nt;
    const bool rec = J->prob.nrec > 0;
    std::vector<JobOp> &ops = J->ops;
    const std::vector<Action> acts = revolve_schedule(nt, J->c.po.nsnap, nullptr);
    std::vector<int> slot_time(std::max(J->c.po.nsnap, 1), -1);
    auto fwd = [&](int a, int b, int record) {
        if (a < b) ops.push_back(JobOp{JOP_FWD, a, b, 0, record});
    };
    int cur = 0;
    size_t i = 0;
    for (; i < acts.size() && acts[i].op != OP_ADJOINT; ++i) {   // recording sweep
        const Action &a = acts[i];
        if (a.op == OP_ADVANCE) {
            fwd(cur, a.arg, 1);
            cur = a.arg;
        } else if (a.op == OP_TAKESHOT) {
            ops.push_back(JobOp{JOP_SNAP, cur, 0, a.arg, 0});
            slot_time[a.arg] = cur;
        }
    }
    fwd(cur, nt, 1);
    if (rec) ops.push_back(JobOp{JOP_GATHER, nt, 0, 0, 0});
    ops.push_back(JobOp{JOP_MISFIT, 0, 0, 0, 0});
    ops.push_back(JobOp{JOP_ZERO_ADJ, 0, 0, 0, 0});
    ops.push_back(JobOp{JOP_ADJ, nt, nt, 0, 0});
    cur = nt;
    for (; i < acts.size(); ++i) {   // reversal
        const Action &a = acts[i];
        switch (a.op) {
        case OP_ADJOINT: ops.push_back(JobOp{JOP_ADJ, a.arg, a.arg, 0, 0}); break;
        case OP_ADVANCE: fwd(cur, a.arg, 0); cur = a.arg; break;
        case OP_TAKESHOT:
            ops.push_back(JobOp{JOP_SNAP, cur, 0, a.arg, 0});
            slot_time[a.arg] = cur;
            break;
        case OP_RESTORE:
            cur = slot_time[a.arg];
            ops.push_back(JobOp{JOP_RESTORE, cur, 0, a.arg, 0});
            break;
        case OP_RESTART: ops.push_back(JobOp{JOP_ZERO_STATE, 0, 0, 0, 0}); cur = 0; break;
        default: break;
        }
    }
    ops.push_back(JobOp{JOP_FOLD, 0, 0, 0, 0});
}

// Program of a job: step ranges (split into chunks by fwi_jobs_advance) and
// the per-job operations between them, for the job's checkpoint policy.
void build_program(fwi_job *J)
{
    const int nt = J->prob.nt;
    const bool rec = J->prob.nrec > 0;
    std::vector<JobOp> &ops = J->ops;
    auto fwd = [&](int a, int b, int record) {
        if (a < b) ops.push_back(JobOp{JOP_FWD, a, b, 0, record});
    };
    auto adj = [&](int hi, int lo) {
        if (hi >= lo) ops.push_back(JobOp{JOP_ADJ, hi, lo, 0, 0});
    };
    if (J->kind == 0) {   // forward
        fwd(0, nt, 1);
        if (rec) ops.push_back(JobOp{JOP_GATHER, nt, 0, 0, 0});
        return;
    }
    if (J->c.po.kind == FWI_CKPT_REVOLVE) {
        build_revolve_program(J);
        return;
    }
    const int K = J->c.po.every, ctop = J->c.po.ctop;
    for (int s = 0; s < nt; s += K) {
        const int e = std::min(nt, s + K);
        fwd(s, e, 1);
        if (e % K == 0 && e <= ctop - K) ops.push_back(JobOp{JOP_SNAP, e, 0, e / K - 1, 0});
    }
    if (rec) ops.push_back(JobOp{JOP_GATHER, nt, 0, 0, 0});
    ops.push_back(JobOp{JOP_MISFIT, 0, 0, 0, 0});
    ops.push_back(JobOp{JOP_ZERO_ADJ, 0, 0, 0, 0});
    adj(nt, std::max(ctop, 1));
    for (int base = ctop - K; base >= 0; base -= K) {
        if (base == 0) ops.push_back(JobOp{JOP_ZERO_STATE, 0, 0, 0, 0});
        else ops.push_back(JobOp{JOP_RESTORE, base, 0, base / K - 1, 0});
        if (K > 1) fwd(base, base + K - 1, 0);
        adj(base + K - 1, std::max(base, 1));
    }
    ops.push_back(JobOp{JOP_FOLD, 0, 0, 0, 0});
}

}  // namespace

// ----------------------------------------------------------------- the ABI
extern "C" {

const char *fwi_strerror(int status)
{
    switch (status) {
    case FWI_OK: return "ok";
    case FWI_EINVAL: return "invalid argument";
    case FWI_ECFL: return "time step above the stability limit";
    case FWI_EBOUNDS: return "position outside the model grid";
    case FWI_ENOMEM: return "workspace too small";
    case FWI_EHIP: return "HIP runtime error";
    case FWI_ENONFINITE: return "non-finite wavefield or misfit";
    case FWI_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char *fwi_last_error(void) { return g_err; }

int fwi_cfl_limit(int32_t ndim, int32_t order, double *h_cfl_max)
{
    if (ndim != 2 && ndim != 3) return fail(FWI_EINVAL, "ndim must be 2 or 3");
    if (order != 2 && order != 4 && order != 8 && order != 16)
        return fail(FWI_EINVAL, "order must be 2, 4, 8 or 16");
    if (!h_cfl_max) return fail(FWI_EINVAL, "NULL output");
    *h_cfl_max = std::sqrt(4.0 / (ndim * max_symbol(order)));
    return FWI_OK;
}

int fwi_workspace_bytes(const fwi_problem *prob, int32_t mode, const fwi_ckpt *ckpt,
                        uint64_t *h_bytes)
{
    if (!h_bytes) return fail(FWI_EINVAL, "NULL output");
    if (mode < FWI_MODE_FORWARD || mode > FWI_MODE_CKPT_BUF) return fail(FWI_EINVAL, "bad mode");
    Geometry g;
    int st = make_geometry(prob, &g);
    if (st) return st;
    Policy po;
    const int m = mode == FWI_MODE_CKPT_BUF ? FWI_MODE_FORWARD_CKPT : mode;
    st = make_policy(prob, g, m, ckpt, &po);
    if (st) return st;
    Layout L;
    make_layout(prob, g, po, m, &L);
    *h_bytes = mode == FWI_MODE_CKPT_BUF ? L.ck_total : L.ws_total;
    return FWI_OK;
}

int fwi_forward(const fwi_problem *prob, const float *v, const float *src,
                const int32_t *src_pos, const int32_t *rec_pos, float *traces, void *ws,
                uint64_t ws_bytes, void *stream)
{
    try {
        Ctx c;
        int st = prepare(c, prob, FWI_MODE_FORWARD, nullptr, ws, ws_bytes, nullptr, 0, stream);
        if (st) return st;
        if (!src || (prob->nrec > 0 && !traces)) return fail(FWI_EINVAL, "NULL input/output array");
        st = stage(c, v, src, src_pos, rec_pos, prob->nrec > 0 ? traces : nullptr, nullptr, 0);
        if (st) return st;
        st = forward_phase(c, prob->nrec > 0);
        if (st) return st;
        return check_level(c, prob->nt);
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_forward_noalloc(const fwi_problem *prob, const float *v, const float *src,
                        const int32_t *src_pos, const int32_t *rec_pos, float *traces,
                        void *stream)
{
    uint64_t need = 0;
    int st = fwi_workspace_bytes(prob, FWI_MODE_FORWARD, nullptr, &need);
    if (st) return st;
    if (need > kScratchBytes)
        return fail(FWI_ENOMEM,
                    "fwi_forward_noalloc: the problem needs %llu workspace bytes, more than the "
                    "fixed %llu-byte workspace (use fwi_forward)",
                    (unsigned long long)need, (unsigned long long)kScratchBytes);
    void *ws = nullptr;
    if (scratch_address(&ws) != 0)
        return fail(FWI_EHIP, "fwi_forward_noalloc: no address for the fixed workspace");
    return fwi_forward(prob, v, src, src_pos, rec_pos, traces, ws, kScratchBytes, stream);
}

int fwi_forward_ckpt(const fwi_problem *prob, const float *v, const float *src,
                     const int32_t *src_pos, const int32_t *rec_pos, const fwi_ckpt *ckpt,
                     float *traces, void *ckpt_buf, uint64_t ckpt_bytes, void *ws,
                     uint64_t ws_bytes, void *stream)
{
    try {
        Ctx c;
        int st = prepare(c, prob, FWI_MODE_FORWARD_CKPT, ckpt, ws, ws_bytes, ckpt_buf,
                         ckpt_bytes, stream);
        if (st) return st;
        if (!src || (prob->nrec > 0 && !traces)) return fail(FWI_EINVAL, "NULL input/output array");
        st = stage(c, v, src, src_pos, rec_pos, prob->nrec > 0 ? traces : nullptr, nullptr, 1);
        if (st) return st;
        st = forward_phase(c, prob->nrec > 0);
        if (st) return st;
        return check_level(c, prob->nt);
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_backward(const fwi_problem *prob, const float *v, const float *src,
                 const int32_t *src_pos, const int32_t *rec_pos, const fwi_ckpt *ckpt,
                 void *ckpt_buf, uint64_t ckpt_bytes, const float *grad_traces, float *dv,
                 void *ws, uint64_t ws_bytes, void *stream)
{
    try {
        Ctx c;
        int st = prepare(c, prob, FWI_MODE_BACKWARD, ckpt, ws, ws_bytes, ckpt_buf, ckpt_bytes,
                         stream);
        if (st) return st;
        if (!src || !dv || (prob->nrec > 0 && !grad_traces))
            return fail(FWI_EINVAL, "NULL input/output array");
        st = stage(c, v, src, src_pos, rec_pos, nullptr, grad_traces, 1);
        if (st) return st;
        st = backward_phase(c);
        if (st) return st;
        st = fold(c, v, dv);
        if (st) return st;
        return check_model(c, dv);
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_gradient(const fwi_problem *prob, const float *v, const float *src,
                 const int32_t *src_pos, const int32_t *rec_pos, const float *obs,
                 const fwi_ckpt *ckpt, double *h_misfit, float *dv, float *traces_or_null,
                 void *ws, uint64_t ws_bytes, void *stream)
{
    try {
        Ctx c;
        int st = prepare(c, prob, FWI_MODE_GRADIENT, ckpt, ws, ws_bytes, nullptr, 0, stream);
        if (st) return st;
        if (!src || !dv || !h_misfit || (prob->nrec > 0 && !obs))
            return fail(FWI_EINVAL, "NULL input/output array");
        float *res = c.f_at(c.L.res, true);
        float *rec = traces_or_null ? traces_or_null : res;
        st = stage(c, v, src, src_pos, rec_pos, prob->nrec > 0 ? rec : nullptr, res, 1);
        if (st) return st;
        st = forward_phase(c, prob->nrec > 0);
        if (st) return st;
        double *d_mis = reinterpret_cast<double *>(c.ws + c.L.misfit);
        const int64_t ntr = (int64_t)prob->nshots * prob->nt * prob->nrec;
        if (ntr > 0) {
            launch_misfit(rec, obs, res, ntr, reinterpret_cast<double *>(c.ws + c.L.partial),
                          d_mis, c.st);
        } else {
            launch_fill(reinterpret_cast<float *>(d_mis), 4, 0.f, c.st);   // 16 B slot
        }
        HIP_TRY(hipGetLastError());
        st = backward_phase(c);
        if (st) return st;
        st = fold(c, v, dv);
        if (st) return st;
        HIP_TRY(hipMemcpyAsync(h_misfit, d_mis, sizeof(double), hipMemcpyDeviceToHost, c.st));
        HIP_TRY(hipStreamSynchronize(c.st));
        if (!std::isfinite(*h_misfit)) return fail(FWI_ENONFINITE, "misfit is not finite");
        return check_model(c, dv);
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_velocity_range(const float *v, int64_t n, float *h_vmin, float *h_vmax, void *ws,
                       uint64_t ws_bytes, void *stream)
{
    if (!v || n < 1 || !h_vmin || !h_vmax || !ws) return fail(FWI_EINVAL, "bad argument");
    const int B = vstats_blocks();
    if (ws_bytes < 4096 || ws_bytes < sizeof(float) * 3ull * B)
        return fail(FWI_ENOMEM, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    float *d = static_cast<float *>(ws);
    launch_vstats(v, n, d, st);
    HIP_TRY(hipGetLastError());
    std::vector<float> h(3 * (size_t)B);
    HIP_TRY(hipMemcpyAsync(h.data(), d, h.size() * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    float lo = INFINITY, hi = -INFINITY, bad = 0.f;
    for (int i = 0; i < B; ++i) {
        lo = std::min(lo, h[i]);
        hi = std::max(hi, h[B + i]);
        bad += h[2 * B + i];
    }
    if (bad > 0.f) return fail(FWI_EINVAL, "velocity has non-finite values");
    *h_vmin = lo;
    *h_vmax = hi;
    return FWI_OK;
}

int fwi_stream_probe(const float *a, const float *b, const float *c, float *out, int64_t n,
                     int32_t variant, void *stream)
{
    if (!a || !b || !c || !out) return fail(FWI_EINVAL, "NULL array");
    if (n < 4 || n % 4 != 0) return fail(FWI_EINVAL, "n must be a positive multiple of 4");
    if (variant < 0 || variant > 15 || (variant & 3) == 3) return fail(FWI_EINVAL, "bad variant");
    const uintptr_t al = reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                         reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(out);
    if (al & 15) return fail(FWI_EINVAL, "arrays must be 16-byte aligned");
    launch_stream_probe(a, b, c, out, n, variant, static_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return FWI_OK;
}

int fwi_tile_probe(const float *cur, const float *prv, const float *kap, float *out, int nz,
                   int ny, int nx, int zc, int32_t mode, int32_t *h_zc, void *stream)
{
    if (!cur || !prv || !kap || !out) return fail(FWI_EINVAL, "NULL field");
    if (out == cur || out == prv || out == kap) return fail(FWI_EINVAL, "out must be distinct");
    if (nz < 1 || ny < 1 || nx < 1 || nz > (1 << 20) || ny > (1 << 20) || nx > (1 << 20))
        return fail(FWI_EINVAL, "grid %d x %d x %d out of range", nz, ny, nx);
    if (zc < 0) return fail(FWI_EINVAL, "zc must be >= 0");
    if (mode < 0 || mode > 9) return fail(FWI_EINVAL, "mode must be 0..9");
    Geometry g;
    g.ndim = 3;
    g.M = 4;
    g.gy = 4;
    g.nz = nz;
    g.ny = ny;
    g.nx = nx;
    g.pitch = (int)align_up((uint64_t)nx + 8, 64);
    g.nya = ny + 8;
    g.plane = (int64_t)g.nya * g.pitch;
    if (g.plane * (int64_t)sizeof(float) >= (int64_t(1) << 31))
        return fail(FWI_EINVAL, "plane too large for 32-bit offsets");
    if (zc == 0) {
        int ntx = 0, nty = 0, nzc = 0;
        tiles_for(g, 1, false, &ntx, &nty, &nzc, &zc);
    }
    zc = std::min(zc, nz);
    if (h_zc) *h_zc = zc;
    launch_tile_probe(cur, prv, kap, out, nz, ny, nx, g.pitch, zc, mode,
                      static_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return FWI_OK;
}

int fwi_revolve_schedule(int32_t nsteps, int32_t slots, int32_t *h_actions, int64_t cap,
                         int64_t *h_count, int64_t *h_forward_steps)
{
    if (nsteps < 1 || slots < 0) return fail(FWI_EINVAL, "nsteps >= 1 and slots >= 0 required");
    if (!h_count || !h_forward_steps) return fail(FWI_EINVAL, "NULL output");
    try {
        int64_t steps = 0;
        std::vector<Action> acts = revolve_schedule(nsteps, slots, &steps);
        *h_count = (int64_t)acts.size();
        *h_forward_steps = steps + 1;   // plus the recording sweep's last step
        if (h_actions)
            for (int64_t i = 0; i < cap && i < (int64_t)acts.size(); ++i) {
                h_actions[2 * i] = acts[i].op;
                h_actions[2 * i + 1] = acts[i].arg;
            }
        return FWI_OK;
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_revolve_plan(int32_t nsteps, int32_t slots, int32_t *h_ops, int64_t cap,
                     int64_t *h_count)
{
    if (nsteps < 1 || slots < 0) return fail(FWI_EINVAL, "nsteps >= 1 and slots >= 0 required");
    if (!h_count || (cap > 0 && !h_ops)) return fail(FWI_EINVAL, "NULL output");
    try {
        fwi_problem p{};
        p.nt = nsteps;
        p.nshots = 1;
        Ctx c;
        c.p = &p;
        c.po.kind = FWI_CKPT_REVOLVE;
        c.po.R = 2;
        c.po.nsnap = std::min(slots, nsteps);
        c.jobs.assign(1, Job{});
        std::vector<int32_t> ops;
        c.plan = &ops;
        int st = forward_phase(c, false);
        if (st) return st;
        st = backward_phase(c);
        if (st) return st;
        *h_count = (int64_t)ops.size() / 10;
        for (int64_t i = 0; i < cap * 10 && i < (int64_t)ops.size(); ++i) h_ops[i] = ops[i];
        return FWI_OK;
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

// Checkpoint policy of a gradient job: as given, or every `chunk` steps.
fwi_ckpt job_ckpt(int32_t chunk, const fwi_ckpt *ckpt)
{
    if (ckpt) return *ckpt;
    fwi_ckpt ck{};
    ck.kind = FWI_CKPT_EVERY;
    ck.every = chunk;
    return ck;
}

int fwi_job_bytes(const fwi_problem *prob, int32_t kind, int32_t chunk, const fwi_ckpt *ckpt,
                  uint64_t *h_bytes)
{
    if (kind != FWI_JOB_FORWARD && kind != FWI_JOB_GRADIENT) return fail(FWI_EINVAL, "bad job kind");
    if (chunk < 1) return fail(FWI_EINVAL, "chunk must be >= 1");
    if (prob && prob->nshots != 1) return fail(FWI_EINVAL, "a job is one shot");
    const fwi_ckpt ck = job_ckpt(chunk, ckpt);
    return fwi_workspace_bytes(prob, kind == FWI_JOB_FORWARD ? FWI_MODE_FORWARD : FWI_MODE_GRADIENT,
                               &ck, h_bytes);
}

int fwi_job_create(const fwi_problem *prob, int32_t kind, int32_t chunk, const fwi_ckpt *ckpt,
                   const float *v, const float *src, const int32_t *src_pos,
                   const int32_t *rec_pos, const float *obs, float *traces, float *dv,
                   void *mem, uint64_t mem_bytes, void *stream, fwi_job **h_job)
{
    if (!h_job) return fail(FWI_EINVAL, "NULL output");
    *h_job = nullptr;
    if (kind != FWI_JOB_FORWARD && kind != FWI_JOB_GRADIENT) return fail(FWI_EINVAL, "bad job kind");
    if (chunk < 1) return fail(FWI_EINVAL, "chunk must be >= 1");
    if (!prob || prob->nshots != 1) return fail(FWI_EINVAL, "a job is one shot");
    try {
        std::unique_ptr<fwi_job> J(new fwi_job());
        J->prob = *prob;
        J->kind = kind;
        J->chunk = chunk;
        const fwi_ckpt ck = job_ckpt(chunk, ckpt);
        const int mode = kind == FWI_JOB_FORWARD ? FWI_MODE_FORWARD : FWI_MODE_GRADIENT;
        Ctx &c = J->c;
        int st = prepare(c, &J->prob, mode, &ck, mem, mem_bytes, nullptr, 0, stream);
        if (st) return st;
        const bool rec = prob->nrec > 0;
        if (!src || (rec && kind == FWI_JOB_FORWARD && !traces)) return fail(FWI_EINVAL, "NULL array");
        if (kind == FWI_JOB_GRADIENT && (!dv || (rec && !obs))) return fail(FWI_EINVAL, "NULL array");
        J->v = v;
        J->obs = obs;
        J->dv = dv;
        if (kind == FWI_JOB_GRADIENT) {
            J->res = c.f_at(c.L.res, true);
            J->d_misfit = reinterpret_cast<double *>(c.ws + c.L.misfit);
            J->rec = traces ? traces : J->res;
        } else {
            J->rec = traces;
        }
        st = stage(c, v, src, src_pos, rec_pos, rec ? J->rec : nullptr, J->res,
                   kind == FWI_JOB_GRADIENT);
        if (st) return st;
        // frames of every level; levels 0 and -1 whole (the job's program
        // also clears them before its first step)
        zero_frames(c, c.jobs[0].ring, (uint64_t)c.po.R);
        zero(c.jobs[0].ring, (uint64_t)c.g.fstride, c.st);
        zero(c.jobs[0].ring + (uint64_t)c.g.fstride * (c.po.R - 1), (uint64_t)c.g.fstride, c.st);
        HIP_TRY(hipGetLastError());
        J->rounds = kind == FWI_JOB_GRADIENT && c.po.kind == FWI_CKPT_REVOLVE;
        build_program(J.get());
        *h_job = J.release();
        return FWI_OK;
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

// Launch groups of one advance: one per (dimension, order, direction, block
// shape); 2-D jobs use two shapes, so at most 4 orders x 2 directions x
// (2 + 1) = 24 groups.
constexpr int kMaxGroups = 24;

int fwi_jobs_ws_bytes(int32_t njobs, int32_t ksteps, uint64_t *h_bytes)
{
    if (njobs < 0 || ksteps < 1 || !h_bytes) return fail(FWI_EINVAL, "bad argument");
    // per group: a job table, two prefix arrays and the level lists of the
    // jobs stepping by rounds (at most one per job and group, ksteps each)
    *h_bytes = kMaxGroups * (align_up(sizeof(Job) * (uint64_t)njobs, kAlign) +
                             align_up(sizeof(int) * 2ull * (njobs + 1), kAlign) +
                             align_up(sizeof(int32_t) * (uint64_t)njobs * ksteps, kAlign)) +
               kAlign;
    return FWI_OK;
}

namespace {

// One job's part of a chunk when it steps by rounds: the direction and level
// of its step in each round (0: none, 1: forward, 2: adjoint), the per-job
// operations due before each round (before[ksteps]: after the last), and
// whether its forward steps record traces.
struct RoundPlan {
    std::vector<int> dir, lev;
    std::vector<std::vector<JobOp>> before;
    int record = -1;
    int used = 0;
};

// Takes up to ksteps steps from the head of J's program, the operations
// between them and the ones right after.  Stops early where the recording
// flag of its forward steps changes (one flag per launch entry).
void plan_rounds(fwi_job *J, int ksteps, RoundPlan &P)
{
    P.dir.assign(ksteps, 0);
    P.lev.assign(ksteps, kNoLevel);
    P.before.assign(ksteps + 1, {});
    int j = 0;
    while (J->head < J->ops.size()) {
        JobOp &o = J->ops[J->head];
        if (!is_step(o)) {
            P.before[j].push_back(o);
            ++J->head;
            continue;
        }
        if (j == ksteps) break;
        if (o.type == JOP_FWD) {
            const int rec = o.record ? 1 : 0;
            if (P.record >= 0 && rec != P.record) break;
            P.record = rec;
            while (o.a < o.b && j < ksteps) { P.dir[j] = 1; P.lev[j] = o.a++; ++j; }
            if (o.a >= o.b) ++J->head;
        } else {
            while (o.a >= o.b && j < ksteps) { P.dir[j] = 2; P.lev[j] = o.a--; ++j; }
            if (o.a < o.b) ++J->head;
        }
    }
    P.used = j;
}

int run_ops(fwi_job *J, const std::vector<JobOp> &ops)
{
    for (const JobOp &o : ops) TRY(run_immediate(J, o));
    return FWI_OK;
}

}  // namespace

int fwi_jobs_advance(fwi_job *const *jobs, int32_t njobs, int32_t ksteps, void *ws,
                     uint64_t ws_bytes, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs) || ksteps < 1) return fail(FWI_EINVAL, "bad argument");
    uint64_t need = 0;
    fwi_jobs_ws_bytes(njobs, ksteps, &need);
    if (!ws || ws_bytes < need) return fail(FWI_ENOMEM, "advance workspace too small");
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0)
        return fail(FWI_EINVAL, "workspace must be 256-byte aligned");
    try {
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (int i = 0; i < njobs; ++i) {
            if (!jobs[i]) return fail(FWI_EINVAL, "NULL job");
            jobs[i]->c.st = st;
        }
        // 1. operations due before this chunk's steps (jobs stepping by
        // rounds run theirs from their round plan)
        for (int i = 0; i < njobs; ++i)
            if (!jobs[i]->rounds) TRY(run_immediates(jobs[i]));
        // 2. gather this chunk's steps into launch groups
        struct Entry {
            const Job *src;   // the job's own table entry (device)
            int32_t win[7];   // n0, k0, fwd_lo, fwd_hi, adj_lo, adj_hi, record
            int levoff;       // level list in the group's lists (-1: none)
        };
        struct Group {
            int ndim = 0, M = 0, adj = 0, nw = 4, steps = 0;
            std::vector<Entry> table;
            std::vector<int> tp{0}, gp{0};
            std::vector<int32_t> lev;   // level lists, ksteps per entry that has one
            Job *d_jobs = nullptr;
            int *d_prefix = nullptr;
            int32_t *d_lev = nullptr;
            int gthreads = 64;
        };
        std::vector<Group> groups;
        auto group_of = [&](int ndim, int M, int adj, int nw) -> Group & {
            for (Group &g : groups)
                if (g.ndim == ndim && g.M == M && g.adj == adj && g.nw == nw) return g;
            groups.push_back(Group{});
            Group &g = groups.back();
            g.ndim = ndim; g.M = M; g.adj = adj; g.nw = nw;
            return g;
        };
        auto add = [&](fwi_job *J, bool isadj, const Entry &e, int steps, bool record,
                       const int32_t *lev) {
            const Job &t = J->c.jobs[0];
            Group &g = group_of(J->c.g.ndim, J->c.g.M, isadj, isadj ? J->c.nw_adj : J->c.nw);
            g.steps = std::max(g.steps, steps);
            g.gthreads = J->c.gthreads;
            Entry x = e;
            if (lev) {
                x.levoff = (int)g.lev.size();
                g.lev.insert(g.lev.end(), lev, lev + ksteps);
            }
            g.table.push_back(x);
            g.tp.push_back(g.tp.back() + t.tile[isadj ? 1 : 0].ntiles);
            g.gp.push_back(g.gp.back() + ((!isadj && record) || isadj ? t.ngather : 0));
        };
        std::vector<RoundPlan> plans(njobs);
        for (int i = 0; i < njobs; ++i) {
            fwi_job *J = jobs[i];
            const Job &t = J->c.jobs[0];
            if (J->rounds) {
                RoundPlan &P = plans[i];
                plan_rounds(J, ksteps, P);
                const bool record = P.record == 1 && J->rec;
                for (int d = 1; d <= 2; ++d) {
                    std::vector<int32_t> lev(ksteps, kNoLevel);
                    int last = 0;
                    for (int j = 0; j < P.used; ++j)
                        if (P.dir[j] == d) { lev[j] = P.lev[j]; last = j + 1; }
                    if (!last) continue;
                    Entry e{J->c.d_jobs, {0, 0, 0, J->prob.nt, 1, J->prob.nt + 1,
                                          d == 1 && record ? 1 : 0}, -1};
                    add(J, d == 2, e, last, d == 1 && record, lev.data());
                }
                continue;
            }
            if (J->head >= J->ops.size()) continue;
            JobOp &o = J->ops[J->head];
            Entry e{J->c.d_jobs, {t.n0, t.k0, t.fwd_lo, t.fwd_hi, t.adj_lo, t.adj_hi, t.record},
                    -1};
            int steps;
            bool record = false;
            if (o.type == JOP_FWD) {
                steps = std::min(ksteps, o.b - o.a);
                record = o.record && J->rec;
                e.win[0] = o.a;
                e.win[2] = o.a;
                e.win[3] = o.a + steps;
                e.win[6] = record ? 1 : 0;
                o.a += steps;
            } else {
                steps = std::min(ksteps, o.a - o.b + 1);
                e.win[1] = o.a;
                e.win[5] = o.a + 1;
                e.win[4] = o.a - steps + 1;
                o.a -= steps;
            }
            const bool finished = o.type == JOP_FWD ? o.a >= o.b : o.a < o.b;
            if (finished) ++J->head;
            add(J, o.type == JOP_ADJ, e, steps, record, nullptr);
        }
        if ((int)groups.size() > kMaxGroups) return fail(FWI_EINVAL, "internal: too many launch groups");
        // 3. assemble the tables on the device (kernel arguments carry them:
        // no host copy to wait for; the stream orders them after the previous
        // chunk's launches, which read the same workspace) and launch every
        // step of the chunk for all groups
        char *w = static_cast<char *>(ws);
        uint64_t off = 0;
        for (Group &g : groups) {
            const int n = (int)g.table.size();
            g.d_jobs = reinterpret_cast<Job *>(w + off);
            off += align_up(sizeof(Job) * (uint64_t)n, kAlign);
            g.d_prefix = reinterpret_cast<int *>(w + off);
            off += align_up(sizeof(int) * 2ull * (n + 1), kAlign);
            g.d_lev = reinterpret_cast<int32_t *>(w + off);
            off += align_up(sizeof(int32_t) * g.lev.size(), kAlign);
            if (off > ws_bytes) return fail(FWI_EINVAL, "internal: advance workspace layout");
            std::vector<int> pre(g.tp);
            pre.insert(pre.end(), g.gp.begin(), g.gp.end());
            const int np = (int)pre.size(), nl = (int)g.lev.size();
            for (int j0 = 0, p0 = 0, l0 = 0; j0 < n || p0 < np || l0 < nl;) {
                AssembleArgs a{};
                a.first = j0;
                a.count = std::min(kAssembleJobs, n - j0);
                for (int k = 0; k < a.count; ++k) {
                    a.src[k] = g.table[j0 + k].src;
                    std::copy(g.table[j0 + k].win, g.table[j0 + k].win + 7, a.win[k]);
                    a.levoff[k] = g.table[j0 + k].levoff;
                }
                a.pfirst = p0;
                a.nprefix = std::min(kAssemblePrefix, np - p0);
                std::copy(pre.begin() + p0, pre.begin() + p0 + a.nprefix, a.prefix);
                a.lfirst = l0;
                a.nlev = std::min(kAssembleLevels, nl - l0);
                std::copy(g.lev.begin() + l0, g.lev.begin() + l0 + a.nlev, a.lev);
                launch_assemble(a, g.d_jobs, g.d_prefix, g.d_lev, st);
                j0 += a.count;
                p0 += a.nprefix;
                l0 += a.nlev;
            }
        }
        HIP_TRY(hipGetLastError());
        for (int j = 0; j < ksteps; ++j) {
            // per-job operations between this job's rounds (snapshot and
            // restore copies of binomial checkpointing), in stream order
            for (int i = 0; i < njobs; ++i)
                if (jobs[i]->rounds) TRY(run_ops(jobs[i], plans[i].before[j]));
            for (Group &g : groups) {
                if (j >= g.steps) continue;
                const int n = (int)g.table.size();
                const int ttiles = g.tp.back(), gblocks = g.gp.back();
                launch_step(g.ndim, g.M, g.nw, g.adj != 0, g.d_jobs, g.d_prefix, n, j, ttiles,
                            g.adj ? 0 : gblocks, 1, LevelMap{}, st);
                if (g.adj && g.ndim == 3)   // 2-D steps add the adjoint source themselves
                    launch_adj_inject(g.d_jobs, g.d_prefix + n + 1, n, gblocks, g.gthreads, j, st);
            }
        }
        HIP_TRY(hipGetLastError());
        // 4. operations due right after this chunk (final gather, residual, fold)
        for (int i = 0; i < njobs; ++i) {
            if (jobs[i]->rounds) TRY(run_ops(jobs[i], plans[i].before[ksteps]));
            else TRY(run_immediates(jobs[i]));
        }
        HIP_TRY(hipGetLastError());
        return FWI_OK;
    } catch (const std::bad_alloc &) {
        return fail(FWI_EINVAL, "host allocation failed");
    } catch (...) {
        return fail(FWI_EINVAL, "internal error");
    }
}

int fwi_job_query(const fwi_job *job, int32_t *h_done, int64_t *h_steps_left)
{
    if (!job) return fail(FWI_EINVAL, "NULL job");
    int64_t steps = 0;
    for (size_t i = job->head; i < job->ops.size(); ++i) {
        const JobOp &o = job->ops[i];
        if (o.type == JOP_FWD) steps += std::max(0, o.b - o.a);
        else if (o.type == JOP_ADJ) steps += std::max(0, o.a - o.b + 1);
    }
    if (h_done) *h_done = job->head == job->ops.size();
    if (h_steps_left) *h_steps_left = steps;
    return FWI_OK;
}

int fwi_job_misfit(const fwi_job *job, double *h_misfit, void *stream)
{
    if (!job || !h_misfit) return fail(FWI_EINVAL, "bad argument");
    if (job->kind != FWI_JOB_GRADIENT) return fail(FWI_EINVAL, "not a gradient job");
    if (job->head < job->ops.size()) return fail(FWI_EINVAL, "job not finished");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(h_misfit, job->d_misfit, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return FWI_OK;
}

int fwi_job_misfit_device(const fwi_job *job, const double **d_misfit)
{
    if (!job || !d_misfit) return fail(FWI_EINVAL, "bad argument");
    if (job->kind != FWI_JOB_GRADIENT) return fail(FWI_EINVAL, "not a gradient job");
    *d_misfit = job->d_misfit;
    return FWI_OK;
}

void fwi_job_destroy(fwi_job *job) { delete job; }

}  // extern "C"
