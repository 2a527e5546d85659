// fwi_kernels.hip -- gfx950 kernels of the acoustic FWI hot path.
//
// One launch of a step kernel advances every job of a job table by one time
// step (Eq. 3 of the paper with a sponge; star Laplacian of Fig. 3):
//     out = alpha * (2 p + kappa' * L'p + src) - beta * p_prev
// with L'p = sum_m c_m [(p_{+m} - p) + (p_{-m} - p)] summed over the axes
// (the Laplacian times dx^2; radius 1 evaluated in this difference form for
// fp32 accuracy, the outer radii as plain sums) and kappa' = (v dt / dx)^2.  The adjoint launch applies the same operator to
// the scaled adjoint field psi' (psi = kappa*alpha*lambda, divided by dx^2),
// for which the discrete adjoint recurrence IS the forward recurrence, and
// accumulates the imaging condition g += psi'^{k+1} * L'p^k.  The adjoint
// source enters at the receiver cells: inside the step in 2-D, by a launch
// after each step in 3-D.
//
// Design for CDNA4 (the paper's MXU band-matrix formulation does not apply:
// the star stencil is banded, not a dense contraction, and the step is HBM
// bound at 16 algorithmic bytes per cell-update):
//  * 3-D: 256-thread blocks own a 64 (x) x 16 (y) column of the grid (64 x 8
//    at 16th order and in the adjoint) over a chunk of z planes.  Each thread
//    keeps a register queue of 2M+1 planes for the z-derivative (z marching),
//    the current xy plane with its M-cell halo is staged in LDS for the x and
//    y derivatives, and each thread owns 4 (or 2) consecutive y rows so
//    y-neighbours are reused from LDS.
//  * 2-D: one wavefront per block, 64 columns marching down a chunk of rows.
//  * Each wavefront reads and writes whole aligned 256-byte row segments.
//  * Blocks are remapped so that each XCD (one L2 each) gets a contiguous
//    range of tiles: neighbouring tiles share their halos in the same L2.
//  * Receiver sampling of level n is done by extra blocks of the launch that
//    computes level n+1 (level n is read-only there), so it costs no launch.
//  * Forward level L is field L mod R of the job's ring unless the launch's
//    level map places it in a snapshot field: binomial checkpointing then
//    reads restored states and writes snapshot states in place, without
//    copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fwi_internal.h"

namespace fwi {

// ----------------------------------------------------------------- weights
// Maximal-order central second-derivative weights:
//   c_m = 2 (-1)^{m+1} (M!)^2 / (m^2 (M-m)! (M+m)!)   (difference form: c_0 unused)
__host__ __device__ constexpr double factd(int n) { return n <= 1 ? 1.0 : double(n) * factd(n - 1); }
__host__ __device__ constexpr double weightd(int M, int m)
{
    return 2.0 * ((m & 1) ? 1.0 : -1.0) * factd(M) * factd(M) /
           (double(m) * double(m) * factd(M - m) * factd(M + m));
}
template <int M>
struct Weights {
    float c[M + 1];
    float t3[M + 1], t2[M + 1];   // -6 resp. -4 times sum_{m > k} c_m
    __host__ __device__ constexpr Weights() : c(), t3(), t2()
    {
        for (int m = 1; m <= M; ++m) c[m] = float(weightd(M, m));
        for (int k = 0; k <= M; ++k) {
            double t = 0.0;
            for (int m = k + 1; m <= M; ++m) t += weightd(M, m);
            t3[k] = float(-6.0 * t);
            t2[k] = float(-4.0 * t);
        }
    }
};

// Radius 1, which carries most of the weight (c_1 = 1.6 of sum |c_m| = 1.83
// at 8th order), is summed in difference form (p_{+1} - p) + (p_{-1} - p),
// exact for neighbouring values of similar size.  The outer radii add plain
// neighbour sums and one -2 D (sum_{m>1} c_m) p term: half the arithmetic,
// and their rounding (about 6 eps |p| times their small weights) stays below
// that of radius 1.  Measured against the FP64 oracle, every parity case
// keeps its error within a factor of two of the all-difference form, and
// the 16th-order step runs 19 % faster.  FWI_DIFF_RADII at build time sets
// another number of difference-form radii (99: all).
#ifndef FWI_DIFF_RADII
#define FWI_DIFF_RADII 1
#endif
constexpr int kDiffRadii = FWI_DIFF_RADII;

// ----------------------------------------------------------------- helpers
__device__ __forceinline__ int sponge_depth(int i, int n, int nb)
{
    // cells into the sponge along one axis: max(nb - i, i - (n - 1 - nb), 0)
    return max(max(nb - i, i - (n - 1 - nb)), 0);
}

__device__ __forceinline__ int find_job(const int *__restrict__ prefix, int njobs, int b)
{
    int lo = 0, hi = njobs;   // prefix[lo] <= b < prefix[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Blocks are dealt round-robin to the 8 XCDs; give XCD k the k-th contiguous
// eighth of the tile range instead (a bijection on [0, T)).
__device__ __forceinline__ int xcd_remap(int b, int T)
{
    const int q = T >> 3, r = T & 7, k = b & 7, i = b >> 3;
    return k * q + min(k, r) + i;
}

__device__ __forceinline__ int mod_pos(int a, int R) { int m = a % R; return m < 0 ? m + R : m; }

// Time level a launch's step updates for job J: n0 + step (forward) or
// k0 - step (adjoint), or, for jobs that change direction within a chunk
// (binomial checkpointing in the serving path), the step's entry of the job's
// level list (kNoLevel: no step of this launch's direction in that round).
__device__ __forceinline__ int step_level(const Job *__restrict__ J, int step, bool adj)
{
    // The list entry is block-uniform, but the compiler cannot see that through
    // a global load; without readfirstlane every plane base and buffer
    // resource derived from it would be built lane by lane (waterfall loops,
    // 20 % slower steps).
    if (J->lev) return __builtin_amdgcn_readfirstlane(J->lev[step]);
    return adj ? J->k0 - step : J->n0 + step;
}

// Field of forward level L: the ring slot L mod R, or a snapshot field the
// level map names (block-uniform, scalar).
__device__ __forceinline__ float *level_ptr(const Job *__restrict__ J, const LevelMap &lm, int L)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (lm.lev[i] == L) return J->snap + (int64_t)lm.fld[i] * J->fstride;
    return J->ring + (int64_t)mod_pos(L, J->R) * J->fstride;
}

// Receiver sampling: traces[n-1][r] = p^n[rec_r] (level n is read-only here).
__device__ __forceinline__ void gather_block(const Job *__restrict__ J, const LevelMap &lm, int r,
                                             int n)
{
    if (!J->record || n < 1 || n > J->nt || r >= J->nrec) return;
    const float *cur = level_ptr(J, lm, n);
    J->traces[(int64_t)(n - 1) * J->nrec + r] = cur[J->rec_off[r]];
}

// Adjoint source at receiver r (the first of its cell): the sum of
// res[k-1] over the receivers sharing the cell, in index order, so the
// result is deterministic.  psi'^k gains kappa' times it (alpha = 1 on the
// model grid, where every receiver sits).
__device__ __forceinline__ float adj_source(const Job *__restrict__ J, int k, int r)
{
    const float *res = J->res + (int64_t)(k - 1) * J->nrec;
    float s = res[r];
    for (int q = J->rec_next[r]; q >= 0; q = J->rec_next[q]) s += res[q];
    return s;
}

// Sponge factors from the squared depth d2 = sum_a d_a^2 into the sponge:
// eta dt = eta_dt * d2, alpha = 1/(1 + eta dt), beta = (1 - eta dt) alpha.
// out = alpha * val - beta * prev, written as alpha * (val - (1 - e) prev).
__device__ __forceinline__ float leapfrog(float val, float prev, int d2, float eta_dt)
{
    if (d2 == 0) return val - prev;
    const float e = eta_dt * (float)d2;
    return __builtin_amdgcn_rcpf(1.f + e) * fmaf(-(1.f - e), prev, val);
}

// Streams read or written once per launch (kappa', the previous level, the
// new level, the gradient accumulator) are non-temporal, leaving L2 to the
// rows that neighbouring tiles share (+4 % on the 3-D forward step; keeping
// kappa' or the new level cached instead, for reuse by the next step from the
// Infinity Cache, measured no faster).  FWI_STREAM_CACHED at build time
// restores ordinary accesses.
// Field pointers come from the job table, so the compiler cannot see that
// they address global memory; without the cast every access would be a
// flat load (64-bit address arithmetic per access, and flat loads also hold
// the LDS counter, so each LDS wait would wait for the prefetches too).
#define GMEM __attribute__((address_space(1)))
typedef GMEM float gfloat;

__device__ __forceinline__ const gfloat *gptr(const float *p) { return (const gfloat *)p; }
__device__ __forceinline__ gfloat *gptr(float *p) { return (gfloat *)p; }

// Plane accesses go through a buffer resource (base and size of one plane in
// scalar registers) and a 32-bit per-lane byte offset: no per-lane address
// arithmetic, and an offset past the plane reads zero instead of faulting.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit buffer, CDNA
constexpr int kCacheNT = 2;              // non-temporal cache policy

__device__ __forceinline__ rsrc_t plane_rsrc(const gfloat *f, int zmem, int64_t plane,
                                             int pbytes)
{
    const float *p = (const float *)(f + (int64_t)zmem * plane);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), 0, pbytes, kRsrcWord3);
}
__device__ __forceinline__ float ldb(rsrc_t r, uint32_t boff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, 0));
}
__device__ __forceinline__ float ldb_stream(rsrc_t r, uint32_t boff)
{
#ifdef FWI_STREAM_CACHED
    return ldb(r, boff);
#else
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(r, (int)boff, 0, kCacheNT));
#endif
}
__device__ __forceinline__ void stb_stream(rsrc_t r, uint32_t boff, float v)
{
#ifdef FWI_STREAM_CACHED
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)boff, 0, 0);
#else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)boff, 0,
                                          kCacheNT);
#endif
}

// Plane of a field: element (z, row, col) is at base[(z + M) * plane + row_offset].
// The plane base is uniform across the block (scalar registers); per-thread
// offsets within a plane are 32-bit, so every load is base + 32-bit offset.
__device__ __forceinline__ const gfloat *plane_ptr(const gfloat *f, int zmem, int64_t plane)
{
    return f + (int64_t)zmem * plane;
}
__device__ __forceinline__ gfloat *plane_ptr(gfloat *f, int zmem, int64_t plane)
{
    return f + (int64_t)zmem * plane;
}

// Compile-time loop: f(Int<I>{}) for I = B .. E-1, fully unrolled, so an
// index derived from I can select a register.
template <int V>
struct Int {
    static constexpr int value = V;
};
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(Int<B>{});
        static_for<B + 1, E>(f);
    }
}

// Byte offset past every plane: a buffer store to it is dropped by the
// hardware's range check, so masked lanes need no branch around a store.
constexpr uint32_t kDropOffset = 0x7ffffff0u;

// Block barrier for LDS traffic only.  __syncthreads() is a workgroup fence
// over all memory, so each wave first waits for every global load it has in
// flight; a step kernel's prefetches for the next plane would then have to
// arrive within the current plane.  The step kernels share nothing through
// global memory within a launch (a cell's previous level, output and
// gradient are read and written by the thread that owns it), so ordering
// the LDS staging is enough.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// --------------------------------------------------------------- 3-D step
// One block: NW wavefronts of RY rows each, a 64 (x) x NW*RY (y) tile,
// marching a chunk of z.  Per plane z: the LDS buffer (z & 1) holds plane z of the propagated field
// with an M-cell halo; registers hold the z-queue (planes z-M .. z+M, in a
// ring indexed by the unrolled phase k, so no register moves), kappa' and
// the previous level.  While plane z is computed, plane z+1 is already being
// loaded (the next queue front, kappa', previous level, halos), and written
// to the other LDS buffer afterwards: one barrier per plane.
//
// Step modes: the forward step; the adjoint step with the imaging condition
// fused in (two stencil fields); and the adjoint as two single-field passes,
// the psi update alone and the imaging condition g += psi^{k+1} * L'p^k
// alone, each with the forward step's memory pattern (see launch_3d).
enum StepMode { kFwd = 0, kAdj = 1, kAdjPsi = 2, kImage = 3 };

// Planes a step kernel loads ahead of the one it computes (queue front,
// kappa', previous level).  Two planes ahead measured no faster on the
// 304^3 forward: 86.7 against 85.1 us per step with 4 x 4 blocks (211
// registers), 85.9 with 4 x 2.  No launch bound caps the registers: one
// wave per SIMD more spills (4 x 4 forward at 3 waves: 98 against 85 us;
// fused adjoint at 4 waves: 190 against 171 us).
template <int M, int MODE>
constexpr int kLookahead = 1;

template <int M, int MODE, int NW, int RY>
__global__ __launch_bounds__(64 * NW) void k_step3d(const Job *__restrict__ jobs,
                                                const int *__restrict__ prefix, int njobs,
                                                int step, int ttiles, int remap, LevelMap lm)
{
    constexpr int TX = kTileX, TY = RY * NW, NT = 64 * NW;
    constexpr int LX = TX + 2 * M, LY = TY + 2 * M, Q = 2 * M + 1, LS = LY * LX;
    constexpr int NYH = (2 * M * TX + NT - 1) / NT;   // y-halo cells per thread
    constexpr int NXH = (TY * 2 * M + NT - 1) / NT;   // x-halo cells per thread
    constexpr bool ADJ = MODE != kFwd;     // adjoint time order and tiling
    constexpr bool FUSED = MODE == kAdj;   // second stencil field (p^k) and g
    constexpr bool IMG = MODE == kImage;
    // single-field modes up to 8th order: halos travel with the queue front
    // (loaded at plane z+M, the same iteration in which the neighbouring tiles
    // load those rows as their own front, so the second read is an L2 hit)
    // and wait in a register ring.  At 16th order the ring would hold 5 x 17
    // values per thread; without it the step runs at 4 instead of 2 waves per
    // SIMD and 46 % faster (122 vs 178 us on a 304^3 grid), while at 8th order
    // the ring wins (89 vs 94 us).
    constexpr bool HQ = !FUSED && M <= 4;
    constexpr Weights<M> W{};
    constexpr int KD = kDiffRadii < M ? kDiffRadii : M;   // radii in difference form
    __shared__ float sp[2 * LS];
    __shared__ float sf[FUSED ? 2 * LS : 1];

    const int tid = threadIdx.x;
    int b = blockIdx.x;
    if (b >= ttiles) {   // receiver-sampling blocks (forward launches only)
        if constexpr (ADJ) return;
        const int gb = b - ttiles;
        const int j = find_job(prefix + njobs + 1, njobs, gb);
        const Job *J = jobs + j;
        gather_block(J, lm, (gb - prefix[njobs + 1 + j]) * blockDim.x + tid, step_level(J, step, false));
        return;
    }
    if (remap) b = xcd_remap(b, ttiles);
    const int j = find_job(prefix, njobs, b);
    const Job *__restrict__ J = jobs + j;
    const int n = step_level(J, step, ADJ);
    if (ADJ ? (n < J->adj_lo || n >= J->adj_hi) : (n < J->fwd_lo || n >= J->fwd_hi)) return;

    const int nz = J->nz, ny = J->ny, nx = J->nx, pitch = J->pitch, nb = J->nb;
    const int64_t plane = J->plane, fstride = J->fstride;
    const Job::Tiling &T = J->tile[ADJ ? 1 : 0];
    int local = b - prefix[j];
    int tx, ty, tz;
    if (T.flags & kTileZFast) {
        tz = local % T.nzc;
        local /= T.nzc;
        tx = local % T.ntx;
        ty = local / T.ntx;
    } else {
        tx = local % T.ntx;
        local /= T.ntx;
        ty = local % T.nty;
        tz = local / T.nty;
    }
    const int z0 = tz * T.zc, z1 = min(z0 + T.zc, nz);
    // marching direction: plane i of the chunk (i = 0 .. npl-1) is zs + dir * i
    const int dir = (T.flags & kTileZAlt) && (tz & 1) ? -1 : 1;
    const int zs = dir > 0 ? z0 : z1 - 1, npl = z1 - z0;

    // cur: the stencil field; prv and kap: the two pointwise streams; out.
    // Imaging mode: cur = p^k, prv = psi^{k+1}, kap = out = g.
    const gfloat *cur, *prv, *kap = gptr(J->kappa);
    gfloat *out;
    const gfloat *fwd = nullptr;
    gfloat *grad = nullptr;
    const bool accum = ADJ && J->accumulate && n <= J->nt - 1;
    if constexpr (IMG) {
        if (!accum) return;
        cur = gptr(level_ptr(J, lm, n));
        prv = gptr(J->adj) + (int64_t)((n + 1) & 1) * fstride;
        kap = gptr(J->grad);
        out = gptr(J->grad);
    } else if constexpr (ADJ) {
        cur = gptr(J->adj) + (int64_t)((n + 1) & 1) * fstride;
        prv = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        out = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        if constexpr (FUSED) {
            fwd = gptr(level_ptr(J, lm, n));
            grad = gptr(J->grad);
        }
    } else {
        cur = gptr(level_ptr(J, lm, n));
        prv = gptr(level_ptr(J, lm, n - 1));
        out = gptr(level_ptr(J, lm, n + 1));
    }
    const float eta_dt = J->eta_dt;
    const int pbytes = (int)(plane * (int64_t)sizeof(float));

    // ---- per-thread geometry (loop invariant)
    const int lane = tid & 63, wv = tid >> 6;
    const int col = tx * TX + lane;   // memory column
    const int x = col - M;            // padded-grid x
    const bool ax = x >= 0 && x < nx;
    // Loads are unconditional: a row past the frame is clamped to the last
    // frame row and a column outside the row to its edge.  Both hold zeros
    // (frames and row padding are zero-filled and never written), exactly
    // the values a masked load would give, and no active cell reads them
    // beyond that.  Stores stay masked.
    const int last_row = ny + 2 * M - 1;   // memory rows per plane - 1
    bool act[RY];
    uint32_t roff[RY];   // byte offsets within a plane
    uint32_t soff[RY];   // store offsets: kDropOffset for cells outside the grid
    int dxy2[RY];
    const int dxs = sponge_depth(x, nx, nb);
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const int yy = ty * TY + wv * RY + i;
        act[i] = ax && yy < ny;
        roff[i] = 4u * (uint32_t)(min(yy + M, last_row) * pitch + col);
        soff[i] = act[i] ? roff[i] : kDropOffset;
        const int d = sponge_depth(yy, ny, nb);
        dxy2[i] = d * d + dxs * dxs;
    }
    uint32_t hyo[NYH], hxo[NXH];
    int hyl[NYH], hxl[NXH];
#pragma unroll
    for (int q = 0; q < NYH; ++q) {   // rows above and below the tile
        const int h = tid + NT * q;
        const int r = (h / TX) % (2 * M), c = h % TX;
        const int ly = r < M ? r : r + TY;
        const int yg = ty * TY - M + ly;
        hyo[q] = 4u * (uint32_t)(min(yg + M, last_row) * pitch + tx * TX + c);
        hyl[q] = h < 2 * M * TX ? ly * LX + M + c : -1;
    }
#pragma unroll
    for (int q = 0; q < NXH; ++q) {   // columns left and right of the tile
        const int h = tid + NT * q;
        const int r = (h / (2 * M)) % TY, c = h % (2 * M);
        const int lc = c < M ? c : c + TX;
        const int cm = min(max(tx * TX - M + lc, 0), pitch - 1);
        const int yg = ty * TY + r;
        hxo[q] = 4u * (uint32_t)(min(yg + M, last_row) * pitch + cm);
        hxl[q] = h < TY * 2 * M ? (M + r) * LX + lc : -1;
    }
    // source (forward): the block that owns it adds it at its plane
    const bool src_blk = !ADJ && J->src_x >= tx * TX - M && J->src_x < tx * TX - M + TX &&
                         J->src_y >= ty * TY && J->src_y < ty * TY + TY && J->src_z >= z0 &&
                         J->src_z < z1;
    float srcv = 0.f;
    int src_row = -1;
    if (src_blk && J->src_x == x) {
        const int r = J->src_y - (ty * TY + wv * RY);
        if (r >= 0 && r < RY) { src_row = r; srcv = J->src_scale * J->wavelet[n]; }
    }

    // ---- register queues.  Chunk plane j (j = -M .. npl-1+M, memory plane
    // zs + dir j + M) lives in queue slot (j + M) % U.  While plane ii is
    // computed from slots ii .. ii+2M (mod U), planes up to ii+M+D-1 are
    // already loaded and the front plane ii+M+D is loaded straight into a
    // free slot (U >= Q + D), so no register is copied after a load and the
    // wave never waits for recent prefetches before it moves on.  kappa', the
    // previous level (and g) of plane ii are in slot ii % (D + 1), loaded D
    // planes ahead.  The plane loop is unrolled by U, a multiple of D + 1,
    // so every slot index is a compile-time constant.  Halos staged from
    // memory at the end of a plane (no halo ring) are loaded one plane ahead,
    // first, so that the wait for them leaves the rest in flight.
    constexpr int D = kLookahead<M, MODE>;
    constexpr int P = D + 1;
    constexpr int U = (Q + D + P - 1) / P * P;
    float q[RY][U];
    float f[FUSED ? RY : 1][FUSED ? U : 1];
    float hy[HQ ? NYH : 1][HQ ? U : 1], hx[HQ ? NXH : 1][HQ ? U : 1];
    if constexpr (HQ) {
        // halos of chunk planes 1 .. M+D-1 (slots M+1 .. 2M+D-1)
#pragma unroll
        for (int s = M + 1; s < Q + D - 1; ++s) {
            if (s - M >= npl) continue;
            const rsrc_t ph = plane_rsrc(cur, zs + dir * (s - M) + M, plane, pbytes);
#pragma unroll
            for (int h = 0; h < NYH; ++h) hy[h][s] = ldb(ph, hyo[h]);
#pragma unroll
            for (int h = 0; h < NXH; ++h) hx[h][s] = ldb(ph, hxo[h]);
        }
    }
    // chunk planes -M .. M+D-1 (plane j is first read by the stencil of
    // plane j - M, so planes past the chunk's last plane + M are skipped)
#pragma unroll
    for (int s = 0; s < Q + D - 1; ++s) {
        if (s >= Q && s - 2 * M >= npl) continue;
        const int zm = zs + dir * (s - M) + M;
        const rsrc_t pc = plane_rsrc(cur, zm, plane, pbytes);
        const rsrc_t pf = plane_rsrc(fwd, zm, plane, pbytes);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            q[i][s] = ldb(pc, roff[i]);
            if constexpr (FUSED) f[i][s] = ldb(pf, roff[i]);
        }
    }
    float kv[P][RY], pv[P][RY], gv[FUSED ? P : 1][FUSED ? RY : 1];
    // pointwise streams of planes 1 .. D-1
#pragma unroll
    for (int a = 1; a < D; ++a) {
        if (a >= npl) continue;
        const rsrc_t pk = plane_rsrc(kap, zs + dir * a + M, plane, pbytes);
        const rsrc_t pp = plane_rsrc(prv, zs + dir * a + M, plane, pbytes);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            kv[a][i] = ldb_stream(pk, roff[i]);
            pv[a][i] = ldb_stream(pp, roff[i]);
            if constexpr (FUSED)
                gv[a][i] = accum ? ldb_stream(plane_rsrc(grad, zs + dir * a + M, plane, pbytes), roff[i])
                                 : 0.f;
        }
    }
    {
        const rsrc_t pk = plane_rsrc(kap, zs + M, plane, pbytes);
        const rsrc_t pp = plane_rsrc(prv, zs + M, plane, pbytes);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            kv[0][i] = ldb(pk, roff[i]);
            pv[0][i] = ldb(pp, roff[i]);
            if constexpr (FUSED)
                gv[0][i] = accum ? ldb(plane_rsrc(grad, zs + M, plane, pbytes), roff[i]) : 0.f;
        }
        const rsrc_t pc = plane_rsrc(cur, zs + M, plane, pbytes);
        const rsrc_t pf = plane_rsrc(fwd, zs + M, plane, pbytes);
        float *L = sp;           // LDS buffer i & 1 holds chunk plane i
        float *LF = FUSED ? sf : nullptr;
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            L[(M + wv * RY + i) * LX + M + lane] = q[i][M];
            if constexpr (FUSED) LF[(M + wv * RY + i) * LX + M + lane] = f[i][M];
        }
#pragma unroll
        for (int h = 0; h < NYH; ++h)
            if (hyl[h] >= 0) {
                L[hyl[h]] = ldb(pc, hyo[h]);
                if constexpr (FUSED) LF[hyl[h]] = ldb(pf, hyo[h]);
            }
#pragma unroll
        for (int h = 0; h < NXH; ++h)
            if (hxl[h] >= 0) {
                L[hxl[h]] = ldb(pc, hxo[h]);
                if constexpr (FUSED) LF[hxl[h]] = ldb(pf, hxo[h]);
            }
    }
    lds_barrier();

    // Plane ii of the chunk; k = ii % U selects the slots.  The main loop
    // runs whole groups of U planes that all have a next plane (more), with
    // no branch around a load or store, so the compiler's wait counts stay
    // exact and only LDS waits remain at the barrier; the last group runs
    // with those checks.
    auto step_plane = [&](auto K, const int ii, const bool more, const bool ahead)
        __attribute__((always_inline)) {
            constexpr int k = decltype(K)::value;
            const int z = zs + dir * ii;   // grid plane computed now
            const int c = k % P, cn = (k + D) % P;   // pointwise slots of planes ii, ii+D
            const int fs = (k + Q - 1 + D) % U;      // free queue slot: chunk plane ii+M+D
            // ---- prefetch: halos of plane z+dir staged at the end of this
            // plane (without a halo ring), then the queue front z+dir(1+M)
            // and the pointwise streams of plane z+dir; memory plane = grid
            // plane + M
            float nhy[HQ ? 1 : NYH], nhx[HQ ? 1 : NXH];
            float nfy[FUSED ? NYH : 1], nfx[FUSED ? NXH : 1];
            const int zf = z + dir * (D + M) + M, zn = z + dir + M, za = z + dir * D + M;
            if (more) {
                if constexpr (!HQ) {
                    const rsrc_t ph = plane_rsrc(cur, zn, plane, pbytes);
#pragma unroll
                    for (int h = 0; h < NYH; ++h) nhy[h] = ldb(ph, hyo[h]);
#pragma unroll
                    for (int h = 0; h < NXH; ++h) nhx[h] = ldb(ph, hxo[h]);
                }
                if constexpr (FUSED) {
                    const rsrc_t fh = plane_rsrc(fwd, zn, plane, pbytes);
#pragma unroll
                    for (int h = 0; h < NYH; ++h) nfy[h] = ldb(fh, hyo[h]);
#pragma unroll
                    for (int h = 0; h < NXH; ++h) nfx[h] = ldb(fh, hxo[h]);
                }
            }
            if (ahead) {
                const rsrc_t pq = plane_rsrc(cur, zf, plane, pbytes);
                const rsrc_t pk = plane_rsrc(kap, za, plane, pbytes);
                const rsrc_t pp = plane_rsrc(prv, za, plane, pbytes);
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    q[i][fs] = ldb(pq, roff[i]);
                    kv[cn][i] = ldb_stream(pk, roff[i]);
                    pv[cn][i] = ldb_stream(pp, roff[i]);
                }
                if constexpr (HQ) {
#pragma unroll
                    for (int h = 0; h < NYH; ++h) hy[h][fs] = ldb(pq, hyo[h]);
#pragma unroll
                    for (int h = 0; h < NXH; ++h) hx[h][fs] = ldb(pq, hxo[h]);
                }
                if constexpr (FUSED) {
                    const rsrc_t fq = plane_rsrc(fwd, zf, plane, pbytes);
                    const rsrc_t pg = plane_rsrc(grad, za, plane, pbytes);
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        f[i][fs] = ldb(fq, roff[i]);
                        gv[cn][i] = accum ? ldb_stream(pg, roff[i]) : 0.f;
                    }
                }
            }
            // ---- plane z (queue slot (k + M + m) % U holds plane z + dir m)
            const float *L = sp + (ii & 1) * LS;
            const float *LF = FUSED ? sf + (ii & 1) * LS : nullptr;
            const rsrc_t po = plane_rsrc(out, z + M, plane, pbytes);
            const rsrc_t pg = plane_rsrc(grad, z + M, plane, pbytes);
            const int dz = sponge_depth(z, nz, nb);
            float res[RY];
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                const int ly = M + wv * RY + i, lx = M + lane;
                const float pc = q[i][(k + M) % U];
                float acc = 0.f;
#pragma unroll
                for (int m = M; m > KD; --m) {
                    const float t = (L[ly * LX + lx + m] + L[ly * LX + lx - m]) +
                                    (L[(ly + m) * LX + lx] + L[(ly - m) * LX + lx]) +
                                    (q[i][(k + M + m) % U] + q[i][(k + M - m) % U]);
                    acc = fmaf(W.c[m], t, acc);
                }
                if constexpr (KD < M) acc = fmaf(W.t3[KD], pc, acc);
#pragma unroll
                for (int m = KD; m >= 1; --m) {
                    const float d = ((L[ly * LX + lx + m] - pc) + (L[ly * LX + lx - m] - pc)) +
                                    ((L[(ly + m) * LX + lx] - pc) + (L[(ly - m) * LX + lx] - pc)) +
                                    ((q[i][(k + M + m) % U] - pc) + (q[i][(k + M - m) % U] - pc));
                    acc = fmaf(W.c[m], d, acc);
                }
                // imaging: g + psi^{k+1} * L'p^k (kv holds g, pv psi^{k+1}),
                // the same operation as the fused kernel's
                res[i] = IMG ? fmaf(pv[c][i], acc, kv[c][i]) : fmaf(kv[c][i], acc, 2.f * pc);
            }
            if (src_blk && z == J->src_z) {
#pragma unroll
                for (int i = 0; i < RY; ++i) res[i] += i == src_row ? srcv : 0.f;
            }
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                if constexpr (IMG)
                    stb_stream(po, soff[i], res[i]);
                else
                    stb_stream(po, soff[i], leapfrog(res[i], pv[c][i], dxy2[i] + dz * dz, eta_dt));
            }
            if constexpr (FUSED) {
                if (accum) {
#pragma unroll
                    for (int i = 0; i < RY; ++i) {
                        const int ly = M + wv * RY + i, lx = M + lane;
                        const float fc = f[i][(k + M) % U];
                        float lf = 0.f;
#pragma unroll
                        for (int m = M; m > KD; --m) {
                            const float t = (LF[ly * LX + lx + m] + LF[ly * LX + lx - m]) +
                                            (LF[(ly + m) * LX + lx] + LF[(ly - m) * LX + lx]) +
                                            (f[i][(k + M + m) % U] + f[i][(k + M - m) % U]);
                            lf = fmaf(W.c[m], t, lf);
                        }
                        if constexpr (KD < M) lf = fmaf(W.t3[KD], fc, lf);
#pragma unroll
                        for (int m = KD; m >= 1; --m) {
                            const float d =
                                ((LF[ly * LX + lx + m] - fc) + (LF[ly * LX + lx - m] - fc)) +
                                ((LF[(ly + m) * LX + lx] - fc) + (LF[(ly - m) * LX + lx] - fc)) +
                                ((f[i][(k + M + m) % U] - fc) + (f[i][(k + M - m) % U] - fc));
                            lf = fmaf(W.c[m], d, lf);
                        }
                        stb_stream(pg, soff[i], fmaf(q[i][(k + M) % U], lf, gv[c][i]));
                    }
                }
            }
            // ---- stage plane z+dir in the other LDS buffer
            if (more) {
                float *Ln = sp + ((ii + 1) & 1) * LS;
                float *LFn = FUSED ? sf + ((ii + 1) & 1) * LS : nullptr;
#pragma unroll
                for (int i = 0; i < RY; ++i) {
                    Ln[(M + wv * RY + i) * LX + M + lane] = q[i][(k + M + 1) % U];
                    if constexpr (FUSED)
                        LFn[(M + wv * RY + i) * LX + M + lane] = f[i][(k + M + 1) % U];
                }
#pragma unroll
                for (int h = 0; h < NYH; ++h)
                    if (hyl[h] >= 0) {
                        if constexpr (HQ) Ln[hyl[h]] = hy[h][(k + M + 1) % U];
                        else Ln[hyl[h]] = nhy[h];
                        if constexpr (FUSED) LFn[hyl[h]] = nfy[h];
                    }
#pragma unroll
                for (int h = 0; h < NXH; ++h)
                    if (hxl[h] >= 0) {
                        if constexpr (HQ) Ln[hxl[h]] = hx[h][(k + M + 1) % U];
                        else Ln[hxl[h]] = nhx[h];
                        if constexpr (FUSED) LFn[hxl[h]] = nfx[h];
                    }
            }
            lds_barrier();
    };
    int ib = 0;
    for (; ib + U - 1 + D < npl; ib += U)
        static_for<0, U>([&](auto K) __attribute__((always_inline)) {
            step_plane(K, ib + decltype(K)::value, true, true);
        });
    static_for<0, U>([&](auto K) __attribute__((always_inline)) {
        const int ii = ib + decltype(K)::value;
        if (ii < npl) step_plane(K, ii, ii + 1 < npl, ii + D < npl);
    });
}

// --------------------------------------------------------------- 2-D step
// One wavefront per block: 64 columns marching down a chunk of rows with a
// (2M+1)-row register queue; the current row with its halo is staged in a
// double-buffered LDS row, and row z+1 is loaded while row z is computed.
template <int M, bool ADJ>
__global__ __launch_bounds__(64) void k_step2d(const Job *__restrict__ jobs,
                                               const int *__restrict__ prefix, int njobs,
                                               int step, int ttiles, int remap, LevelMap lm)
{
    constexpr int TX = kTileX, LX = TX + 2 * M, Q = 2 * M + 1;
    constexpr Weights<M> W{};
    constexpr int KD = kDiffRadii < M ? kDiffRadii : M;   // radii in difference form
    __shared__ float sp[2 * LX];
    __shared__ float sf[ADJ ? 2 * LX : 1];
    __shared__ float sinj[ADJ ? TX : 1];   // adjoint source of the current row

    const int lane = threadIdx.x;
    int b = blockIdx.x;
    if (b >= ttiles) {
        if constexpr (ADJ) return;
        const int gb = b - ttiles;
        const int j = find_job(prefix + njobs + 1, njobs, gb);
        const Job *J = jobs + j;
        gather_block(J, lm, (gb - prefix[njobs + 1 + j]) * blockDim.x + lane, step_level(J, step, false));
        return;
    }
    if (remap) b = xcd_remap(b, ttiles);
    const int j = find_job(prefix, njobs, b);
    const Job *__restrict__ J = jobs + j;
    const int n = step_level(J, step, ADJ);
    if (ADJ ? (n < J->adj_lo || n >= J->adj_hi) : (n < J->fwd_lo || n >= J->fwd_hi)) return;

    const int nz = J->nz, nx = J->nx, pitch = J->pitch, nb = J->nb;
    const int64_t fstride = J->fstride;
    const Job::Tiling &T = J->tile[ADJ ? 1 : 0];
    const int local = b - prefix[j];
    const int tx = local % T.ntx;
    const int tz = local / T.ntx;
    const int z0 = tz * T.zc, z1 = min(z0 + T.zc, nz);
    // adjoint: the psi update adds the adjoint source at this tile's receiver
    // cells (a list sorted by row; at most one cell per column)
    int rp = 0, re = 0;
    if constexpr (ADJ) {
        rp = J->rt_start[local];
        re = J->rt_start[local + 1];
    }

    const gfloat *cur, *prv;
    gfloat *out;
    const gfloat *fwd = nullptr;
    gfloat *grad = nullptr;
    bool accum = false;
    if constexpr (ADJ) {
        cur = gptr(J->adj) + (int64_t)((n + 1) & 1) * fstride;
        prv = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        out = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        accum = J->accumulate && n <= J->nt - 1;
        fwd = gptr(level_ptr(J, lm, n));
        grad = gptr(J->grad);
    } else {
        cur = gptr(level_ptr(J, lm, n));
        prv = gptr(level_ptr(J, lm, n - 1));
        out = gptr(level_ptr(J, lm, n + 1));
    }
    const gfloat *kap = gptr(J->kappa);
    const float eta_dt = J->eta_dt;

    const int col = tx * TX + lane;
    const int x = col - M;
    const bool act = x >= 0 && x < nx;
    const int dxs = sponge_depth(x, nx, nb);
    // halo lanes: lane < 2M loads column tx*TX - M + (lane < M ? lane : lane + TX)
    const int hl = lane < M ? lane : lane + TX;
    const int hcol = tx * TX - M + hl;
    const bool hact = lane < 2 * M && hcol >= 0 && hcol < pitch;
    const int hcl = min(max(hcol, 0), pitch - 1);   // a column inside the row
    const bool src_here = !ADJ && J->src_x == x && J->src_z >= z0 && J->src_z < z1;
    const float srcv = src_here ? J->src_scale * J->wavelet[n] : 0.f;
    const int64_t p64 = pitch;

    // Register queue of U = Q + 1 rows: chunk row j (row z0 + j, j = -M ..)
    // in slot (j + M) % U; the front row is loaded straight into the free
    // slot and kappa', the previous level (and g) alternate between two
    // slots, so no freshly loaded register is copied and the wave keeps the
    // next row's loads in flight while it computes (as in the 3-D kernel).
    // Lanes outside the grid load and store zeros in the row's frame and
    // padding, which hold zeros, so stores need no mask.
    constexpr int U = Q + 1;
    float q[U];
    float f[ADJ ? U : 1];
#pragma unroll
    for (int s = 0; s < Q; ++s) {   // rows z0 - M .. z0 + M
        q[s] = act ? cur[(int64_t)(z0 + s) * p64 + col] : 0.f;
        if constexpr (ADJ) f[s] = act ? fwd[(int64_t)(z0 + s) * p64 + col] : 0.f;
    }
    float kv[2], pv[2], gv[2];
    kv[0] = act ? kap[(int64_t)(z0 + M) * p64 + col] : 0.f;
    pv[0] = act ? prv[(int64_t)(z0 + M) * p64 + col] : 0.f;
    gv[0] = 0.f;
    if constexpr (ADJ) gv[0] = act && accum ? grad[(int64_t)(z0 + M) * p64 + col] : 0.f;
    {
        float *L = sp + (z0 & 1) * LX;
        L[M + lane] = q[M];
        if (lane < 2 * M) L[hl] = hact ? cur[(int64_t)(z0 + M) * p64 + hcol] : 0.f;
        if constexpr (ADJ) {
            float *LF = sf + (z0 & 1) * LX;
            LF[M + lane] = f[M];
            if (lane < 2 * M) LF[hl] = hact ? fwd[(int64_t)(z0 + M) * p64 + hcol] : 0.f;
        }
    }
    lds_barrier();

    // row z = z0 + ii; k = ii % U selects the slots
    auto step_row = [&](auto K, const int z, const bool more) __attribute__((always_inline)) {
            constexpr int k = decltype(K)::value;
            const int c = k & 1, cn = c ^ 1;   // pointwise slots of rows z, z+1
            const int fs = (k + U - 1) % U;    // free queue slot: row z+M+1
            // halos of row z+1 (staged at the end of this row) first.  The
            // loads are not predicated (a skipped load would make the wait
            // counts after it inexact): lanes outside the grid read the zero
            // frame and padding of their row, halo lanes a clamped column.
            float nh = 0.f, nfh = 0.f;
            if (more) {
                const int64_t rf = (int64_t)(z + 1 + 2 * M) * p64, rc = (int64_t)(z + 1 + M) * p64;
                const float h = cur[rc + hcl];
                nh = hact ? h : 0.f;
                if constexpr (ADJ) {
                    const float hf = fwd[rc + hcl];
                    nfh = hact ? hf : 0.f;
                }
                q[fs] = cur[rf + col];
                kv[cn] = kap[rc + col];
                pv[cn] = prv[rc + col];
                if constexpr (ADJ) {
                    f[fs] = fwd[rf + col];
                    const float g = grad[rc + col];
                    gv[cn] = accum ? g : 0.f;
                }
            }
            const float *L = sp + (z & 1) * LX;
            const int lx = M + lane;
            const float pc = q[(k + M) % U];
            float acc = 0.f;
#pragma unroll
            for (int m = M; m > KD; --m) {
                const float t = (L[lx + m] + L[lx - m]) + (q[(k + M + m) % U] + q[(k + M - m) % U]);
                acc = fmaf(W.c[m], t, acc);
            }
            if constexpr (KD < M) acc = fmaf(W.t2[KD], pc, acc);
#pragma unroll
            for (int m = KD; m >= 1; --m) {
                const float d = ((L[lx + m] - pc) + (L[lx - m] - pc)) +
                                ((q[(k + M + m) % U] - pc) + (q[(k + M - m) % U] - pc));
                acc = fmaf(W.c[m], d, acc);
            }
            float val = fmaf(kv[c], acc, 2.f * pc);
            if (src_here && z == J->src_z) val += srcv;
            const int dz = sponge_depth(z, nz, nb);
            const int64_t rz = (int64_t)(z + M) * p64 + col;
            float o = leapfrog(val, pv[c], dxs * dxs + dz * dz, eta_dt);
            if constexpr (ADJ) {
                // receivers on row z: lane i takes the list's i-th, and the sum
                // reaches the lane of its column through LDS
                if (rp < re && (J->rt_key[rp] >> 6) == z) {
                    const int idx = rp + lane;
                    const int key = idx < re ? J->rt_key[idx] : -1;
                    const int r = key >= 0 && (key >> 6) == z ? J->rt_rec[idx] : -1;
                    sinj[lane] = 0.f;
                    lds_barrier();
                    if (r >= 0) sinj[key & 63] = adj_source(J, n, r);
                    lds_barrier();
                    if (act) o += kv[c] * sinj[lane];
                    rp += __popcll(__ballot(r >= 0));
                    lds_barrier();
                }
            }
            out[rz] = o;   // zero outside the grid
            if constexpr (ADJ) {
                if (accum) {
                    const float *LF = sf + (z & 1) * LX;
                    const float fc = f[(k + M) % U];
                    float lf = 0.f;
#pragma unroll
                    for (int m = M; m > KD; --m) {
                        const float t = (LF[lx + m] + LF[lx - m]) + (f[(k + M + m) % U] + f[(k + M - m) % U]);
                        lf = fmaf(W.c[m], t, lf);
                    }
                    if constexpr (KD < M) lf = fmaf(W.t2[KD], fc, lf);
#pragma unroll
                    for (int m = KD; m >= 1; --m) {
                        const float d = ((LF[lx + m] - fc) + (LF[lx - m] - fc)) +
                                        ((f[(k + M + m) % U] - fc) + (f[(k + M - m) % U] - fc));
                        lf = fmaf(W.c[m], d, lf);
                    }
                    grad[rz] = fmaf(pc, lf, gv[c]);   // zero outside the grid
                }
            }
            if (more) {
                float *Ln = sp + ((z + 1) & 1) * LX;
                Ln[M + lane] = q[(k + M + 1) % U];
                if (lane < 2 * M) Ln[hl] = nh;
                if constexpr (ADJ) {
                    float *LFn = sf + ((z + 1) & 1) * LX;
                    LFn[M + lane] = f[(k + M + 1) % U];
                    if (lane < 2 * M) LFn[hl] = nfh;
                }
            }
            lds_barrier();
    };
    int zb = z0;
    for (; zb + U < z1; zb += U)
        static_for<0, U>([&](auto K) __attribute__((always_inline)) {
            step_row(K, zb + decltype(K)::value, true);
        });
    static_for<0, U>([&](auto K) __attribute__((always_inline)) {
        const int z = zb + decltype(K)::value;
        if (z < z1) step_row(K, z, z + 1 < z1);
    });
}

// 2-D step for grids too small to fill the GPU: one block per tile row of 64
// columns and one cell per lane, every neighbour loaded straight from memory
// (the fields are cache-resident at these sizes).  Nothing is marched, so a
// launch costs one round of load latency instead of the 2M + 1 row warm-up
// and serial row loop of k_step2d.  The arithmetic is k_step2d's, term by term
// in the same order, so both kernels give bitwise the same fields.  Tiles are
// one row tall (Tiling.zc == 1); the adjoint takes this row's receiver cells
// from the tile's list, as k_step2d does row by row.
template <int M, bool ADJ>
__global__ __launch_bounds__(64) void k_step2d_direct(const Job *__restrict__ jobs,
                                                      const int *__restrict__ prefix, int njobs,
                                                      int step, int ttiles, int remap,
                                                      LevelMap lm)
{
    constexpr int TX = kTileX;
    constexpr Weights<M> W{};
    constexpr int KD = kDiffRadii < M ? kDiffRadii : M;   // radii in difference form
    __shared__ float sinj[ADJ ? TX : 1];   // adjoint source of this row

    const int lane = threadIdx.x;
    int b = blockIdx.x;
    if (b >= ttiles) {
        if constexpr (ADJ) return;
        const int gb = b - ttiles;
        const int j = find_job(prefix + njobs + 1, njobs, gb);
        const Job *J = jobs + j;
        gather_block(J, lm, (gb - prefix[njobs + 1 + j]) * blockDim.x + lane, step_level(J, step, false));
        return;
    }
    if (remap) b = xcd_remap(b, ttiles);
    const int j = find_job(prefix, njobs, b);
    const Job *__restrict__ J = jobs + j;
    const int n = step_level(J, step, ADJ);
    if (ADJ ? (n < J->adj_lo || n >= J->adj_hi) : (n < J->fwd_lo || n >= J->fwd_hi)) return;

    const int nz = J->nz, nx = J->nx, pitch = J->pitch, nb = J->nb;
    const int64_t fstride = J->fstride;
    const Job::Tiling &T = J->tile[ADJ ? 1 : 0];
    const int local = b - prefix[j];
    const int tx = local % T.ntx;
    const int z = local / T.ntx;   // one row per tile
    if (z >= nz) return;

    const gfloat *cur, *prv;
    gfloat *out;
    const gfloat *fwd = nullptr;
    gfloat *grad = nullptr;
    bool accum = false;
    if constexpr (ADJ) {
        cur = gptr(J->adj) + (int64_t)((n + 1) & 1) * fstride;
        prv = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        out = gptr(J->adj) + (int64_t)(n & 1) * fstride;
        accum = J->accumulate && n <= J->nt - 1;
        fwd = gptr(level_ptr(J, lm, n));
        grad = gptr(J->grad);
    } else {
        cur = gptr(level_ptr(J, lm, n));
        prv = gptr(level_ptr(J, lm, n - 1));
        out = gptr(level_ptr(J, lm, n + 1));
    }
    const gfloat *kap = gptr(J->kappa);
    const float eta_dt = J->eta_dt;

    const int col = tx * TX + lane;
    const int x = col - M;
    const bool act = x >= 0 && x < nx;
    // every neighbour of an active cell lies inside the frame (zeros beyond the
    // padded grid), where k_step2d reads the same values from LDS and its queue
    const int64_t p64 = pitch, rz = (int64_t)(z + M) * p64 + col;
    float o = 0.f, pc = 0.f, kv = 0.f, gv = 0.f, lf = 0.f;
    if (act) {
        pc = cur[rz];
        kv = kap[rz];
        const float pv = prv[rz];
        float acc = 0.f;
#pragma unroll
        for (int m = M; m > KD; --m) {
            const float t = (cur[rz + m] + cur[rz - m]) + (cur[rz + m * p64] + cur[rz - m * p64]);
            acc = fmaf(W.c[m], t, acc);
        }
        if constexpr (KD < M) acc = fmaf(W.t2[KD], pc, acc);
#pragma unroll
        for (int m = KD; m >= 1; --m) {
            const float d = ((cur[rz + m] - pc) + (cur[rz - m] - pc)) +
                            ((cur[rz + m * p64] - pc) + (cur[rz - m * p64] - pc));
            acc = fmaf(W.c[m], d, acc);
        }
        float val = fmaf(kv, acc, 2.f * pc);
        // the source term rounded as in k_step2d: its product first, then the
        // sum (never fused into one fma)
        if (!ADJ && J->src_x == x && J->src_z == z) {
#pragma clang fp contract(off)
            const float srcv = J->src_scale * J->wavelet[n];
            val = val + srcv;
        }
        const int dxs = sponge_depth(x, nx, nb), dz = sponge_depth(z, nz, nb);
        o = leapfrog(val, pv, dxs * dxs + dz * dz, eta_dt);
        if constexpr (ADJ) {
            if (accum) {
                gv = grad[rz];
                const float fc = fwd[rz];
#pragma unroll
                for (int m = M; m > KD; --m) {
                    const float t = (fwd[rz + m] + fwd[rz - m]) + (fwd[rz + m * p64] + fwd[rz - m * p64]);
                    lf = fmaf(W.c[m], t, lf);
                }
                if constexpr (KD < M) lf = fmaf(W.t2[KD], fc, lf);
#pragma unroll
                for (int m = KD; m >= 1; --m) {
                    const float d = ((fwd[rz + m] - fc) + (fwd[rz - m] - fc)) +
                                    ((fwd[rz + m * p64] - fc) + (fwd[rz - m * p64] - fc));
                    lf = fmaf(W.c[m], d, lf);
                }
            }
        }
    }
    if constexpr (ADJ) {
        // receivers on this row: lane i takes the list's i-th, and the sum
        // reaches the lane of its column through LDS (block-uniform branch)
        const int rp = J->rt_start[local], re = J->rt_start[local + 1];
        if (rp < re) {
            const int idx = rp + lane;
            const int key = idx < re ? J->rt_key[idx] : -1;
            const int r = key >= 0 ? J->rt_rec[idx] : -1;
            sinj[lane] = 0.f;
            __syncthreads();
            if (r >= 0) sinj[key & 63] = adj_source(J, n, r);
            __syncthreads();
            o += kv * sinj[lane];
        }
    }
    if (act) {
        out[rz] = o;
        if constexpr (ADJ) {
            if (accum) grad[rz] = fmaf(pc, lf, gv);
        }
    }
}

// ------------------------------------------------------------ side kernels
// kappa' = (v dt/dx)^2 on the padded grid (edge-replicated model), 0 on the frame.
__global__ void k_prep_kappa(const float *__restrict__ v, float *__restrict__ kappa,
                             int M, int gy, int nz, int ny, int nx, int pitch, int nya,
                             int nb, int nzm, int nym, int nxm, int64_t total, float dt_dx)
{
    const int64_t plane = (int64_t)nya * pitch;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t zi = idx / plane;
        const int64_t rem = idx - zi * plane;
        const int yi = (int)(rem / pitch), ci = (int)(rem % pitch);
        const int z = (int)zi - M, y = yi - gy, x = ci - M;
        float out = 0.f;
        if (z >= 0 && z < nz && y >= 0 && y < ny && x >= 0 && x < nx) {
            const int zm = min(max(z - nb, 0), nzm - 1);
            const int ym = min(max(y - nb, 0), nym - 1);
            const int xm = min(max(x - nb, 0), nxm - 1);
            const float t = v[((int64_t)zm * nym + ym) * nxm + xm] * dt_dx;
            out = t * t;
        }
        kappa[idx] = out;
    }
}

__global__ void k_fill(float4 *__restrict__ p, int64_t n4, float val)
{
    const float4 w = make_float4(val, val, val, val);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = w;
}

// Snapshots of a leapfrog state (levels t and t-1) for every job of the table.
// dir 0: level -> snap[slot] (the level where the map puts it); 1: snap[slot]
// -> ring; 2: zero the two levels in the ring (t = 0).  mask bit w selects
// level t - w.
__global__ void k_snapshot(const Job *__restrict__ jobs, int slot, int time, int dir, int mask,
                           LevelMap lm)
{
    const Job *J = jobs + (blockIdx.y >> 1);
    const int which = blockIdx.y & 1;
    if (!((mask >> which) & 1)) return;
    float4 *r = reinterpret_cast<float4 *>(
        dir == 0 ? level_ptr(J, lm, time - which)
                 : J->ring + (int64_t)mod_pos(time - which, J->R) * J->fstride);
    float4 *s = reinterpret_cast<float4 *>(J->snap + (int64_t)(2 * slot + which) * J->fstride);
    if (r == s) return;
    const int64_t n4 = J->fstride / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (dir == 0) s[i] = r[i];
        else if (dir == 1) r[i] = s[i];
        else r[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Several forward steps of a small 2-D grid in one launch (temporal blocking
// for launch-bound grids).  A block loads a region of p^n, p^{n-1} and kappa'
// into LDS that extends the output tile by A = K M cells on every side, then
// advances it kk <= K steps in LDS, each step on a region M cells narrower
// (the apron cells are computed redundantly by neighbouring blocks), and
// stores levels n+kk and n+kk-1 of its output tile.  Cells outside the padded
// grid hold zero and are never updated, as the frame in memory.  Each cell's
// arithmetic is k_step2d_direct's, term by term, so the fields and traces are
// bitwise those of kk single steps.  The launch reads ring slots n, n-1 and
// writes slots n+kk, n+kk-1, which must differ (ring length >= K + 2): no
// block reads what another writes.  Traces of levels n .. n+kk are written by
// the block whose output tile holds the receiver (level n too: a preceding
// single step does not sample the level it produces).
template <int M, int K>
struct Multi2d {
    static constexpr int A = K * M;                     // apron
    static constexpr int RW = 64;                        // region width (one wave per row)
    static constexpr int OX = RW - 2 * A, OZ = 16;       // output tile
    static constexpr int RH = OZ + 2 * A, NR = RW * RH;  // region
    static_assert(OX >= 16, "apron too wide for the region");
};

template <int M, int K>
__global__ __launch_bounds__(1024) void k_step2d_multi(const Job *__restrict__ jobs,
                                                       int tiles_per_job, int ntxm, int step,
                                                       int kk, int record)
{
    using G = Multi2d<M, K>;
    constexpr int A = G::A, RW = G::RW, OX = G::OX, OZ = G::OZ, RH = G::RH, NR = G::NR;
    constexpr int NT = 1024, CPT = (NR + NT - 1) / NT;   // region cells per thread
    constexpr int RPT = 2;                               // receivers resolved per thread
    constexpr Weights<M> W{};
    constexpr int KD = kDiffRadii < M ? kDiffRadii : M;
    __shared__ float s0[NR], s1[NR], sk[NR];

    const int tid = threadIdx.x;
    const int j = blockIdx.x / tiles_per_job, t = blockIdx.x % tiles_per_job;
    const Job *__restrict__ J = jobs + j;
    const int n = step_level(J, step, false);
    const int nz = J->nz, nx = J->nx, pitch = J->pitch, nb = J->nb, nrec = J->nrec;
    const int x0 = (t % ntxm) * OX - A, z0 = (t / ntxm) * OZ - A;   // region origin
    const gfloat *cur = gptr(level_ptr(J, LevelMap{}, n));
    const gfloat *prv = gptr(level_ptr(J, LevelMap{}, n - 1));
    const gfloat *kap = gptr(J->kappa);
    gfloat *o1 = gptr(level_ptr(J, LevelMap{}, n + kk));
    gfloat *o0 = gptr(level_ptr(J, LevelMap{}, n + kk - 1));
    const float eta_dt = J->eta_dt;
    const int64_t p64 = pitch;

    // this thread's region cells: LDS index, grid coordinates, inside the grid
    int ci[CPT], cx[CPT], cz[CPT];
    bool cin[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        ci[q] = tid + q * NT;
        cx[q] = x0 + ci[q] % RW;
        cz[q] = z0 + ci[q] / RW;
        cin[q] = ci[q] < NR && cx[q] >= 0 && cx[q] < nx && cz[q] >= 0 && cz[q] < nz;
    }
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        if (ci[q] >= NR) continue;
        const int64_t off = (int64_t)(cz[q] + M) * p64 + (cx[q] + M);
        s0[ci[q]] = cin[q] ? cur[off] : 0.f;
        s1[ci[q]] = cin[q] ? prv[off] : 0.f;
        sk[ci[q]] = cin[q] ? kap[off] : 0.f;
    }
    // receivers in this block's output tile: their LDS index (-1: elsewhere).
    // Grids on this path are small, so field offsets fit 32 bits.
    const bool rec_on = record && J->record;
    auto local_of = [&](int r) {
        const int off = (int)J->rec_off[r];
        const int rx = off % pitch - M - x0, rz = off / pitch - M - z0;
        return rx >= A && rx < A + OX && rz >= A && rz < A + OZ ? rz * RW + rx : -1;
    };
    int rl[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * NT;
        rl[q] = rec_on && r < nrec ? local_of(r) : -1;
    }
    // traces of level L (1 .. nt) from the LDS field f
    auto sample = [&](const float *f, int L) {
        if (!rec_on || L < 1 || L > J->nt) return;
        float *tr = J->traces + (int64_t)(L - 1) * nrec;
#pragma unroll
        for (int q = 0; q < RPT; ++q)
            if (rl[q] >= 0) tr[tid + q * NT] = f[rl[q]];
        for (int r = tid + RPT * NT; r < nrec; r += NT) {
            const int li = local_of(r);
            if (li >= 0) tr[r] = f[li];
        }
    };
    __syncthreads();
    sample(s0, n);

    float *cu = s0, *pr = s1;   // levels L and L-1; the step writes L+1 over L-1
    for (int st = 0; st < kk; ++st) {
        const int L = n + st, lo = (st + 1) * M;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int i = ci[q], rx = i % RW, rz = i / RW;
            if (!cin[q] || rx < lo || rx >= RW - lo || rz < lo || rz >= RH - lo) continue;
            const int x = cx[q], z = cz[q];
            const float pc = cu[i];
            const float kv = sk[i];
            const float pv = pr[i];
            float acc = 0.f;
#pragma unroll
            for (int m = M; m > KD; --m) {
                const float tt = (cu[i + m] + cu[i - m]) + (cu[i + m * RW] + cu[i - m * RW]);
                acc = fmaf(W.c[m], tt, acc);
            }
            if constexpr (KD < M) acc = fmaf(W.t2[KD], pc, acc);
#pragma unroll
            for (int m = KD; m >= 1; --m) {
                const float d = ((cu[i + m] - pc) + (cu[i - m] - pc)) +
                                ((cu[i + m * RW] - pc) + (cu[i - m * RW] - pc));
                acc = fmaf(W.c[m], d, acc);
            }
            float val = fmaf(kv, acc, 2.f * pc);
            if (J->src_x == x && J->src_z == z) {
#pragma clang fp contract(off)
                const float srcv = J->src_scale * J->wavelet[L];
                val = val + srcv;
            }
            const int dxs = sponge_depth(x, nx, nb), dz = sponge_depth(z, nz, nb);
            pr[i] = leapfrog(val, pv, dxs * dxs + dz * dz, eta_dt);
        }
        __syncthreads();
        float *tmp = cu;
        cu = pr;
        pr = tmp;
        sample(cu, L + 1);
    }

#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const int i = ci[q], rx = i % RW, rz = i / RW;
        if (!cin[q] || rx < A || rx >= A + OX || rz < A || rz >= A + OZ) continue;
        const int64_t off = (int64_t)(cz[q] + M) * p64 + (cx[q] + M);
        o1[off] = cu[i];
        o0[off] = pr[i];
    }
}

// Final receiver sampling (level n = n0 + step).
__global__ void k_gather(const Job *__restrict__ jobs, const int *__restrict__ gprefix,
                         int njobs, int step, LevelMap lm)
{
    const int j = find_job(gprefix, njobs, blockIdx.x);
    const Job *J = jobs + j;
    gather_block(J, lm, (blockIdx.x - gprefix[j]) * blockDim.x + threadIdx.x, J->n0 + step);
}

// Adjoint source of 3-D steps, a launch after each adjoint step: psi'^k[rec]
// += kappa'[rec] * res[k-1][rec] (2-D steps add it themselves).
__global__ void k_adj_inject(const Job *__restrict__ jobs, const int *__restrict__ gprefix,
                             int njobs, int step)
{
    const int j = find_job(gprefix, njobs, blockIdx.x);
    const Job *J = jobs + j;
    const int k = step_level(J, step, true);
    const int r = (blockIdx.x - gprefix[j]) * blockDim.x + threadIdx.x;
    if (k < J->adj_lo || k >= J->adj_hi || r >= J->nrec || !J->rec_head[r]) return;
    const float s = adj_source(J, k, r);
    const int64_t off = J->rec_off[r];
    float *psi = J->adj + (int64_t)(k & 1) * J->fstride;
    psi[off] += J->kappa[off] * s;
}

// Misfit (Eq. 1) and adjoint source: res = 2 (d - obs); per-block partial sums
// of (d - obs)^2 in fp64, reduced in a fixed order (deterministic).
// d and res may be the same array (traces recorded into the residual
// buffer): each element is read and then written by the same thread, and
// neither pointer is declared restrict.
__global__ __launch_bounds__(256) void k_misfit(const float *d, const float *__restrict__ obs,
                                                float *res, int64_t n,
                                                double *__restrict__ partial)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double e = (double)d[i] - (double)obs[i];
        res[i] = (float)(2.0 * e);
        acc += e * e;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partial,
                                                      int n, double *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Transpose of the edge padding, one axis at a time: padded index i of an
// axis of padded length np maps to model index clamp(i - nb, 0, nm - 1).
__device__ __forceinline__ void fold_range(int im, int nm, int np, int nb, int &lo, int &hi)
{
    lo = im == 0 ? 0 : im + nb;
    hi = im == nm - 1 ? np - 1 : im + nb;
}

// x pass: out1[z][y][xm] = sum_shots sum_{x -> xm} g_s(z, y, x)
__global__ void k_fold_x(const Job *__restrict__ jobs, int njobs, int M, int gy,
                         int nxm, float *__restrict__ out1)
{
    const Job *J0 = jobs;
    const int nz = J0->nz, ny = J0->ny, nx = J0->nx, nb = J0->nb, pitch = J0->pitch;
    const int64_t plane = J0->plane;
    const int64_t total = (int64_t)nz * ny * nxm;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int xm = (int)(idx % nxm);
        const int64_t zy = idx / nxm;
        const int y = (int)(zy % ny), z = (int)(zy / ny);
        int lo, hi;
        fold_range(xm, nxm, nx, nb, lo, hi);
        const int64_t base = (int64_t)(z + M) * plane + (int64_t)(y + gy) * pitch + M;
        float s = 0.f;
        for (int jb = 0; jb < njobs; ++jb) {
            const float *g = jobs[jb].grad + base;
            for (int x = lo; x <= hi; ++x) s += g[x];
        }
        out1[idx] = s;
    }
}

// y pass (3-D): out2[z][ym][xm] = sum_{y -> ym} in[z][y][xm]
__global__ void k_fold_y(const float *__restrict__ in, int nz, int ny, int nym, int nxm, int nb,
                         float *__restrict__ out2)
{
    const int64_t total = (int64_t)nz * nym * nxm;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int xm = (int)(idx % nxm);
        const int64_t zy = idx / nxm;
        const int ym = (int)(zy % nym), z = (int)(zy / nym);
        int lo, hi;
        fold_range(ym, nym, ny, nb, lo, hi);
        float s = 0.f;
        for (int y = lo; y <= hi; ++y) s += in[((int64_t)z * ny + y) * nxm + xm];
        out2[idx] = s;
    }
}

// z pass and chain rule: dv[m] = (2 / v[m]) * sum_{z -> zm} in[z][ym][xm]
// (d kappa / d v = 2 kappa / v; the kappa cancels against psi = kappa*alpha*lambda).
__global__ void k_fold_z(const float *__restrict__ in, const float *__restrict__ v, int nz,
                         int nzm, int nym, int nxm, int nb, float *__restrict__ dv)
{
    const int64_t per = (int64_t)nym * nxm;
    const int64_t total = (int64_t)nzm * per;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int zm = (int)(idx / per);
        const int64_t yx = idx - (int64_t)zm * per;
        int lo, hi;
        fold_range(zm, nzm, nz, nb, lo, hi);
        float s = 0.f;
        for (int z = lo; z <= hi; ++z) s += in[(int64_t)z * per + yx];
        dv[idx] = 2.f * s / v[idx];
    }
}

// Model statistics for host validation: per-block min, max and count of
// non-finite velocities (partial[0..nb), [nb..2nb), [2nb..3nb)).
__global__ __launch_bounds__(256) void k_vstats(const float *__restrict__ v, int64_t n,
                                                float *__restrict__ partial)
{
    __shared__ float smin[256], smax[256], sbad[256];
    float lo = INFINITY, hi = -INFINITY, bad = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float a = v[i];
        if (!isfinite(a)) bad += 1.f;
        else { lo = fminf(lo, a); hi = fmaxf(hi, a); }
    }
    smin[threadIdx.x] = lo; smax[threadIdx.x] = hi; sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + s]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + s]);
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = smin[0];
        partial[gridDim.x + blockIdx.x] = smax[0];
        partial[2 * gridDim.x + blockIdx.x] = sbad[0];
    }
}

// --------------------------------------------------- bandwidth ceiling probe
// A pointwise stream with the forward step's memory mix: three fields read,
// one written (out = a + b * c), each field touched once per launch.  Any
// step kernel that reads p, p_prev and kappa' and writes p_next moves at
// least these bytes, so the probe's rate bounds the step's on this chip.
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));

template <typename V, bool NT>
__device__ __forceinline__ V ld_probe(const V *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename V, bool NT>
__device__ __forceinline__ void st_probe(V *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename V, bool NT>
__global__ __launch_bounds__(256) void k_stream3r1w(const V *__restrict__ a,
                                                    const V *__restrict__ b,
                                                    const V *__restrict__ c,
                                                    V *__restrict__ o, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const V x = ld_probe<V, NT>(a + i), y = ld_probe<V, NT>(b + i), z = ld_probe<V, NT>(c + i);
        st_probe<V, NT>(o + i, x + y * z);
    }
}

template <typename V, bool NT>
static void launch_probe_t(const float *a, const float *b, const float *c, float *o, int64_t n,
                           bool persistent, hipStream_t st)
{
    constexpr int W = sizeof(V) / sizeof(float);
    const int64_t nv = n / W;
    const int64_t full = (nv + 255) / 256;
    const int grid = (int)(persistent ? std::min<int64_t>(full, 2048) : full);
    hipLaunchKernelGGL((k_stream3r1w<V, NT>), dim3(grid), dim3(256), 0, st,
                       reinterpret_cast<const V *>(a), reinterpret_cast<const V *>(b),
                       reinterpret_cast<const V *>(c), reinterpret_cast<V *>(o), nv);
}

// variant: bits 0-1 load width (0: 32-bit, 1: 64-bit, 2: 128-bit), bit 2
// non-temporal, bit 3 a grid of at most 2048 blocks striding over the fields
// (otherwise one lane per vector).  n is a multiple of 4.
void launch_stream_probe(const float *a, const float *b, const float *c, float *o, int64_t n,
                         int variant, hipStream_t st)
{
    const bool nt = (variant >> 2) & 1, pers = (variant >> 3) & 1;
    switch (variant & 3) {
    case 0:
        if (nt) launch_probe_t<float, true>(a, b, c, o, n, pers, st);
        else launch_probe_t<float, false>(a, b, c, o, n, pers, st);
        break;
    case 1:
        if (nt) launch_probe_t<vf2, true>(a, b, c, o, n, pers, st);
        else launch_probe_t<vf2, false>(a, b, c, o, n, pers, st);
        break;
    default:
        if (nt) launch_probe_t<vf4, true>(a, b, c, o, n, pers, st);
        else launch_probe_t<vf4, false>(a, b, c, o, n, pers, st);
        break;
    }
}

// ------------------------------------------------ tile-march pattern probe
// The 8th-order forward step's memory pattern with the stencil taken out:
// blocks of 4 wavefronts x 4 rows march 64 x 16 column tiles through z
// chunks in the step's block order (XCD-remapped), load cur, prv and kappa
// once per cell through buffer resources (prv and kappa non-temporal) one
// plane ahead, and write out = 2 cur + kappa prv with the step's store.
// Mode bits add the step's other traffic and synchronisation one at a
// time: 1 the halo rows and columns of cur (loaded one plane ahead, as the
// step's 16th-order kernels and adjoints do), 2 the plane staged in LDS
// behind the LDS-only barrier (the written cur value then comes from LDS),
// 4 the 2M warm-up planes of cur each chunk reads around its own.  Halo and
// warm-up values enter only a sum scaled by `zero` (0 from the host), so
// the output stays 2 cur + kappa prv for finite inputs.
template <int MODE>
__global__ __launch_bounds__(256) void k_tile_probe(const float *cur, const float *prv,
                                                    const float *kap, float *out, int nz, int ny,
                                                    int nx, int pitch, int zc, int ntx, int nty,
                                                    int ttiles, float zero)
{
    constexpr int M = 4, TX = kTileX, RY = 4, NW = 4, TY = RY * NW, NT = 64 * NW;
    constexpr int LX = TX + 2 * M, LY = TY + 2 * M, LS = LX * LY;
    constexpr int NYH = (2 * M * TX + NT - 1) / NT, NXH = (TY * 2 * M + NT - 1) / NT;
    constexpr bool HALO = MODE & 1, LDS = MODE & 2, WARM = MODE & 4;
    __shared__ float sp[LDS ? 2 * LS : 1];
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, ttiles);
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty, tz = b / nty;
    const int z0 = tz * zc, z1 = min(z0 + zc, nz);
    const int64_t plane = (int64_t)(ny + 2 * M) * pitch;
    const int pbytes = (int)(plane * (int64_t)sizeof(float));
    const int lane = tid & 63, wv = tid >> 6;
    const int col = tx * TX + lane, x = col - M;
    const int last_row = ny + 2 * M - 1;
    uint32_t roff[RY], soff[RY];
    int lrow[RY];
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        const int yy = ty * TY + wv * RY + i;
        roff[i] = 4u * (uint32_t)(min(yy + M, last_row) * pitch + col);
        soff[i] = x >= 0 && x < nx && yy < ny ? roff[i] : kDropOffset;
        lrow[i] = (M + wv * RY + i) * LX + M + lane;
    }
    uint32_t hyo[NYH], hxo[NXH];
    int hyl[NYH], hxl[NXH];
#pragma unroll
    for (int q = 0; q < NYH; ++q) {
        const int h = tid + NT * q;
        const int r = (h / TX) % (2 * M), c = h % TX;
        const int ly = r < M ? r : r + TY;
        const int yg = ty * TY - M + ly;
        hyo[q] = 4u * (uint32_t)(min(max(yg + M, 0), last_row) * pitch + tx * TX + c);
        hyl[q] = h < 2 * M * TX ? ly * LX + M + c : -1;
    }
#pragma unroll
    for (int q = 0; q < NXH; ++q) {
        const int h = tid + NT * q;
        const int r = (h / (2 * M)) % TY, c = h % (2 * M);
        const int lc = c < M ? c : c + TX;
        const int cm = min(max(tx * TX - M + lc, 0), pitch - 1);
        hxo[q] = 4u * (uint32_t)(min(ty * TY + r + M, last_row) * pitch + cm);
        hxl[q] = h < TY * 2 * M ? (M + r) * LX + lc : -1;
    }
    float acc = 0.f;
    if constexpr (WARM) {
        // memory planes z0 .. z0+M-1 and z1+M .. z1+2M-1: the M planes on
        // either side of the chunk that the step's z-queue reads
#pragma unroll
        for (int s = 0; s < 2 * M; ++s) {
            const int zm = s < M ? z0 + s : z1 + s;
            const rsrc_t pw = plane_rsrc(gptr(cur), zm, plane, pbytes);
#pragma unroll
            for (int i = 0; i < RY; ++i) acc += ldb(pw, roff[i]);
        }
    }
    // Three-slot rings, chunk plane j in slot j % 3: cur and its halos are
    // loaded two planes ahead, so the plane staged into LDS at the end of an
    // iteration was loaded one iteration earlier (as the step's queue front
    // and halo ring are); kappa and prv one plane ahead.
    float q[3][RY], kv[3][RY], pv[3][RY];
    float hy[3][HALO ? NYH : 1], hx[3][HALO ? NXH : 1];
    auto load_cur = [&](const int sl, const int z) __attribute__((always_inline)) {
        const rsrc_t pc = plane_rsrc(gptr(cur), z + M, plane, pbytes);
        if constexpr (HALO) {
#pragma unroll
            for (int h = 0; h < NYH; ++h) hy[sl][h] = ldb(pc, hyo[h]);
#pragma unroll
            for (int h = 0; h < NXH; ++h) hx[sl][h] = ldb(pc, hxo[h]);
        }
#pragma unroll
        for (int i = 0; i < RY; ++i) q[sl][i] = ldb(pc, roff[i]);
    };
    auto load_pw = [&](const int sl, const int z) __attribute__((always_inline)) {
        const rsrc_t pk = plane_rsrc(gptr(kap), z + M, plane, pbytes);
        const rsrc_t pp = plane_rsrc(gptr(prv), z + M, plane, pbytes);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            kv[sl][i] = ldb_stream(pk, roff[i]);
            pv[sl][i] = ldb_stream(pp, roff[i]);
        }
    };
    // plane z's cells (and halos) into LDS buffer z & 1, or its halos into
    // the sum
    auto stage = [&](const int sl, const int z) __attribute__((always_inline)) {
        if constexpr (LDS) {
            float *L = sp + (z & 1) * LS;
#pragma unroll
            for (int i = 0; i < RY; ++i) L[lrow[i]] = q[sl][i];
            if constexpr (HALO) {
#pragma unroll
                for (int h = 0; h < NYH; ++h)
                    if (hyl[h] >= 0) L[hyl[h]] = hy[sl][h];
#pragma unroll
                for (int h = 0; h < NXH; ++h)
                    if (hxl[h] >= 0) L[hxl[h]] = hx[sl][h];
            }
        } else if constexpr (HALO) {
#pragma unroll
            for (int h = 0; h < NYH; ++h) acc += hy[sl][h];
#pragma unroll
            for (int h = 0; h < NXH; ++h) acc += hx[sl][h];
        }
    };
    load_cur(0, z0);
    if (z0 + 1 < z1) load_cur(1, z0 + 1);
    load_pw(0, z0);
    stage(0, z0);
    if constexpr (LDS) lds_barrier();
    // plane z (chunk slot K): loads of z+2 (cur) and z+1 (kappa, prv), the
    // store of z, then plane z+1 staged
    auto step_plane = [&](auto K, const int z, const bool more1, const bool more2)
        __attribute__((always_inline)) {
        constexpr int c = decltype(K)::value, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        if (more2) load_cur(c2, z + 2);
        if (more1) load_pw(c1, z + 1);
        const rsrc_t po = plane_rsrc(gptr(out), z + M, plane, pbytes);
        const float extra = zero * acc;
        const float *L = sp + (z & 1) * LS;
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            const float cv = LDS ? L[lrow[i]] : q[c][i];
            stb_stream(po, soff[i], fmaf(kv[c][i], pv[c][i], 2.f * cv) + extra);
        }
        if (more1) stage(c1, z + 1);
        if constexpr (LDS) lds_barrier();
    };
    int z = z0;
    for (; z + 5 <= z1; z += 3) {
        step_plane(Int<0>{}, z, true, true);
        step_plane(Int<1>{}, z + 1, true, true);
        step_plane(Int<2>{}, z + 2, true, true);
    }
    static_for<0, 4>([&](auto K) __attribute__((always_inline)) {
        const int zz = z + decltype(K)::value;
        if (zz < z1) step_plane(Int<decltype(K)::value % 3>{}, zz, zz + 1 < z1, zz + 2 < z1);
    });
}

// The bare march (with or without the halo loads) with 64-bit loads and
// stores: each lane owns two adjacent columns of two rows, so one wavefront
// instruction covers two 256-byte row segments.  Same tiles, chunks, block
// order and output as k_tile_probe; halo values enter the zero-scaled sum.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <bool HALO>
__global__ __launch_bounds__(256) void k_tile_probe64(const float *cur, const float *prv,
                                                      const float *kap, float *out, int nz,
                                                      int ny, int nx, int pitch, int zc, int ntx,
                                                      int nty, int ttiles, float zero)
{
    constexpr int M = 4, TX = kTileX, TY = 16;
    const int tid = threadIdx.x;
    int b = xcd_remap(blockIdx.x, ttiles);
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty, tz = b / nty;
    const int z0 = tz * zc, z1 = min(z0 + zc, nz);
    const int64_t plane = (int64_t)(ny + 2 * M) * pitch;
    const int pbytes = (int)(plane * (int64_t)sizeof(float));
    const int lane = tid & 63, wv = tid >> 6;
    const int col = tx * TX + 2 * (lane & 31);   // even: 8-byte aligned
    const int last_row = ny + 2 * M - 1;
    uint32_t roff[2], soff[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int yy = ty * TY + wv * 4 + (lane >> 5) + 2 * i;
        roff[i] = 4u * (uint32_t)(min(yy + M, last_row) * pitch + col);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int x = col + e - M;
            soff[i][e] = x >= 0 && x < nx && yy < ny ? roff[i] + 4u * e : kDropOffset;
        }
    }
    // halos: 8 rows of 64 columns (one pair per thread) and 16 rows of 4 + 4
    // columns (two pairs per row, threads 0..63)
    uint32_t hyo, hxo;
    {
        const int r = tid >> 5, c = 2 * (tid & 31);
        const int ly = r < M ? r : r + TY;
        hyo = 4u * (uint32_t)(min(ty * TY - M + ly + M, last_row) * pitch + tx * TX + c);
        const int xr = (tid >> 2) & 15, xp = tid & 3;
        const int xc = min(max(tx * TX - M + (xp < 2 ? 2 * xp : TX + 2 * xp), 0), pitch - 2);
        hxo = 4u * (uint32_t)(min(ty * TY + xr + M, last_row) * pitch + xc);
    }
    auto ld2 = [&](rsrc_t r, uint32_t off) __attribute__((always_inline)) {
        return __builtin_bit_cast(vf2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    };
    auto ld2_stream = [&](rsrc_t r, uint32_t off) __attribute__((always_inline)) {
        return __builtin_bit_cast(vf2,
                                  __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kCacheNT));
    };
    float acc = 0.f;
    vf2 q[2][2], kv[2][2], pv[2][2], hh[2][2];
    auto load = [&](const int sl, const int z) __attribute__((always_inline)) {
        const rsrc_t pc = plane_rsrc(gptr(cur), z + M, plane, pbytes);
        const rsrc_t pk = plane_rsrc(gptr(kap), z + M, plane, pbytes);
        const rsrc_t pp = plane_rsrc(gptr(prv), z + M, plane, pbytes);
        if constexpr (HALO) {
            hh[sl][0] = ld2(pc, hyo);
            hh[sl][1] = ld2(pc, hxo);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            q[sl][i] = ld2(pc, roff[i]);
            kv[sl][i] = ld2_stream(pk, roff[i]);
            pv[sl][i] = ld2_stream(pp, roff[i]);
        }
    };
    load(0, z0);
    auto step_plane = [&](auto K, const int z, const bool more) __attribute__((always_inline)) {
        constexpr int c = decltype(K)::value, cn = 1 - c;
        if (more) load(cn, z + 1);
        if constexpr (HALO) acc += hh[c][0].x + hh[c][0].y + hh[c][1].x + hh[c][1].y;
        const rsrc_t po = plane_rsrc(gptr(out), z + M, plane, pbytes);
        const float extra = zero * acc;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const vf2 o = {fmaf(kv[c][i].x, pv[c][i].x, 2.f * q[c][i].x) + extra,
                           fmaf(kv[c][i].y, pv[c][i].y, 2.f * q[c][i].y) + extra};
            if (soff[i][0] != kDropOffset && soff[i][1] != kDropOffset)
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, o), po,
                                                      (int)roff[i], 0, kCacheNT);
            else {
                stb_stream(po, soff[i][0], o.x);
                stb_stream(po, soff[i][1], o.y);
            }
        }
    };
    int z = z0;
    for (; z + 2 < z1; z += 2) {
        step_plane(Int<0>{}, z, true);
        step_plane(Int<1>{}, z + 1, true);
    }
    static_for<0, 2>([&](auto K) __attribute__((always_inline)) {
        const int zz = z + decltype(K)::value;
        if (zz < z1) step_plane(K, zz, zz + 1 < z1);
    });
}

// One launch of the tile-march probe over nz x ny x nx cells (8th-order
// frame, rows of `pitch` floats) in z chunks of zc planes.
void launch_tile_probe(const float *cur, const float *prv, const float *kap, float *out, int nz,
                       int ny, int nx, int pitch, int zc, int mode, hipStream_t st)
{
    const int ntx = (nx + 4 + kTileX - 1) / kTileX, nty = (ny + 15) / 16;
    const int nzc = (nz + zc - 1) / zc;
    const int T = ntx * nty * nzc;
    if (mode & 8) {
        if (mode & 1)
            hipLaunchKernelGGL(k_tile_probe64<true>, dim3(T), dim3(256), 0, st, cur, prv, kap,
                               out, nz, ny, nx, pitch, zc, ntx, nty, T, 0.f);
        else
            hipLaunchKernelGGL(k_tile_probe64<false>, dim3(T), dim3(256), 0, st, cur, prv, kap,
                               out, nz, ny, nx, pitch, zc, ntx, nty, T, 0.f);
        return;
    }
    switch (mode & 7) {
#define FWI_TILE_PROBE(m)                                                                     \
    case m:                                                                                   \
        hipLaunchKernelGGL(k_tile_probe<m>, dim3(T), dim3(256), 0, st, cur, prv, kap, out, nz, \
                           ny, nx, pitch, zc, ntx, nty, T, 0.f);                              \
        break;
        FWI_TILE_PROBE(0)
        FWI_TILE_PROBE(1)
        FWI_TILE_PROBE(2)
        FWI_TILE_PROBE(3)
        FWI_TILE_PROBE(4)
        FWI_TILE_PROBE(5)
        FWI_TILE_PROBE(6)
        FWI_TILE_PROBE(7)
#undef FWI_TILE_PROBE
    }
}

// Launch tables of a serving chunk (see AssembleArgs): block i copies entry
// i from the job's memory and patches its time window and level list; block
// 0 also writes the launch's slices of the prefix arrays and level lists.
__global__ __launch_bounds__(64) void k_assemble(AssembleArgs a, Job *__restrict__ table,
                                                 int *__restrict__ prefix,
                                                 int32_t *__restrict__ levels)
{
    const int i = blockIdx.x;
    if (i < a.count) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(a.src[i]);
        uint32_t *dst = reinterpret_cast<uint32_t *>(table + a.first + i);
        constexpr int words = sizeof(Job) / sizeof(uint32_t);
        for (int w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
        __syncthreads();
        if (threadIdx.x == 0) {
            Job &J = table[a.first + i];
            J.n0 = a.win[i][0];
            J.k0 = a.win[i][1];
            J.fwd_lo = a.win[i][2];
            J.fwd_hi = a.win[i][3];
            J.adj_lo = a.win[i][4];
            J.adj_hi = a.win[i][5];
            J.record = a.win[i][6];
            J.lev = a.levoff[i] >= 0 ? levels + a.levoff[i] : nullptr;
        }
    }
    if (i == 0) {
        for (int p = threadIdx.x; p < a.nprefix; p += blockDim.x) prefix[a.pfirst + p] = a.prefix[p];
        for (int p = threadIdx.x; p < a.nlev; p += blockDim.x) levels[a.lfirst + p] = a.lev[p];
    }
}

// Non-finite cells of forward level L of every job (ring slot L mod R):
// per-block counts, partial[0 .. gridDim.x), summed on the host.
__global__ __launch_bounds__(256) void k_nonfinite_level(const Job *__restrict__ jobs, int njobs,
                                                         int L, float *__restrict__ partial)
{
    __shared__ float red[256];
    float bad = 0.f;
    for (int j = 0; j < njobs; ++j) {
        const Job *J = jobs + j;
        const float4 *f =
            reinterpret_cast<const float4 *>(J->ring + (int64_t)mod_pos(L, J->R) * J->fstride);
        const int64_t n4 = J->fstride / 4;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
             i += (int64_t)gridDim.x * blockDim.x) {
            const float4 a = f[i];
            bad += (isfinite(a.x) ? 0.f : 1.f) + (isfinite(a.y) ? 0.f : 1.f) +
                   (isfinite(a.z) ? 0.f : 1.f) + (isfinite(a.w) ? 0.f : 1.f);
        }
    }
    red[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------- fixed per-GPU workspace
// The workspace of fwi_forward_noalloc, for callers that cannot allocate
// device memory: one array per GPU the library runs on, held until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): it looks up each device's own
// address once, with that device current, and passes that address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int scratch_address(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return 0;
}

// ---------------------------------------------------------------- launchers
int vstats_blocks() { return 256; }

void launch_assemble(const AssembleArgs &a, Job *table, int *prefix, int32_t *levels,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_assemble, dim3(a.count > 0 ? a.count : 1), dim3(64), 0, st, a, table,
                       prefix, levels);
}

void launch_nonfinite_level(const Job *jobs, int njobs, int L, float *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_nonfinite_level, dim3(vstats_blocks()), dim3(256), 0, st, jobs, njobs,
                       L, partial);
}

void launch_vstats(const float *v, int64_t n, float *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_vstats, dim3(vstats_blocks()), dim3(256), 0, st, v, n, partial);
}

// The 16th-order adjoint runs as two single-field passes (imaging condition,
// then the psi update): the fused kernel carries two 17-plane queues in
// more registers than fit 2 waves per SIMD, each pass one queue.  Both
// compute bitwise the same values.  At 8th order the fused kernel is as
// fast as the two passes and stays; FWI_SPLIT_ADJ=1 selects the two passes
// there too.
template <int M>
static bool split_adjoint()
{
    if constexpr (M >= 8) {
        return true;
    } else if constexpr (M == 4) {
        const char *e = getenv("FWI_SPLIT_ADJ");
        return e && atoi(e) != 0;
    } else {
        return false;
    }
}

template <int M, int NW, int RY>
static void launch_3d(bool adj, const Job *jobs, const int *prefix, int njobs, int step,
                      int ttiles, int grid, int remap, const LevelMap &lm, hipStream_t st)
{
    const dim3 g(grid), b(64 * NW);
    if (!adj) {
        hipLaunchKernelGGL((k_step3d<M, kFwd, NW, RY>), g, b, 0, st, jobs, prefix, njobs, step,
                           ttiles, remap, lm);
        return;
    }
    if constexpr (M >= 4) {
        if (split_adjoint<M>()) {
            // the imaging pass reads psi^{k+1} and p^k, which the psi pass leaves intact
            hipLaunchKernelGGL((k_step3d<M, kImage, NW, RY>), g, b, 0, st, jobs, prefix, njobs,
                               step, ttiles, remap, lm);
            hipLaunchKernelGGL((k_step3d<M, kAdjPsi, NW, RY>), g, b, 0, st, jobs, prefix, njobs,
                               step, ttiles, remap, lm);
            return;
        }
    }
    if constexpr (M < 8)
        hipLaunchKernelGGL((k_step3d<M, kAdj, NW, RY>), g, b, 0, st, jobs, prefix, njobs, step,
                           ttiles, remap, lm);
}

template <int M, int NW, int RY>
static hipError_t occupancy_3d(int *n, bool adj)
{
    const int t = 64 * NW;
    if (!adj) return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_step3d<M, kFwd, NW, RY>, t, 0);
    if constexpr (M >= 4) {
        if (split_adjoint<M>()) {
            int a = 0, c = 0;
            hipError_t e =
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_step3d<M, kAdjPsi, NW, RY>, t, 0);
            if (e == hipSuccess)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_step3d<M, kImage, NW, RY>, t, 0);
            *n = a < c ? a : c;
            return e;
        }
    }
    if constexpr (M < 8)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_step3d<M, kAdj, NW, RY>, t, 0);
    return hipErrorInvalidValue;
}

template <int M>
static void launch_step_m(int ndim, int nw, bool adj, const Job *jobs, const int *prefix,
                          int njobs, int step, int ttiles, int gblocks, int remap,
                          const LevelMap &lm, hipStream_t st)
{
    const int grid = ttiles + (adj ? 0 : gblocks);
    if (grid <= 0) return;
    if (ndim == 3) {
        switch (nw) {   // wavefronts per block x rows per thread
        case 8: launch_3d<M, 8, 4>(adj, jobs, prefix, njobs, step, ttiles, grid, remap, lm, st); break;
        case 42: launch_3d<M, 4, 2>(adj, jobs, prefix, njobs, step, ttiles, grid, remap, lm, st); break;
        case 82: launch_3d<M, 8, 2>(adj, jobs, prefix, njobs, step, ttiles, grid, remap, lm, st); break;
        default: launch_3d<M, 4, 4>(adj, jobs, prefix, njobs, step, ttiles, grid, remap, lm, st); break;
        }
    } else if (nw == 1) {   // one-row tiles, one cell per lane
        if (adj)
            hipLaunchKernelGGL((k_step2d_direct<M, true>), dim3(grid), dim3(64), 0, st, jobs,
                               prefix, njobs, step, ttiles, remap, lm);
        else
            hipLaunchKernelGGL((k_step2d_direct<M, false>), dim3(grid), dim3(64), 0, st, jobs,
                               prefix, njobs, step, ttiles, remap, lm);
    } else {
        if (adj)
            hipLaunchKernelGGL((k_step2d<M, true>), dim3(grid), dim3(64), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap, lm);
        else
            hipLaunchKernelGGL((k_step2d<M, false>), dim3(grid), dim3(64), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap, lm);
    }
}

// Resident blocks per CU of a step kernel (0 if the query fails).
template <int M>
static int occupancy_m(int ndim, int nw, bool adj)
{
    int n = 0;
    hipError_t e = hipSuccess;
    if (ndim == 3) {
        if (nw == 8) e = occupancy_3d<M, 8, 4>(&n, adj);
        else if (nw == 42) e = occupancy_3d<M, 4, 2>(&n, adj);
        else if (nw == 82) e = occupancy_3d<M, 8, 2>(&n, adj);
        else e = occupancy_3d<M, 4, 4>(&n, adj);
    } else {
        e = adj ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2d<M, true>, 64, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step2d<M, false>, 64, 0);
    }
    return e == hipSuccess ? n : 0;
}

int step_blocks_per_cu(int ndim, int M, int nw, bool adj)
{
    switch (M) {
    case 1: return occupancy_m<1>(ndim, nw, adj);
    case 2: return occupancy_m<2>(ndim, nw, adj);
    case 4: return occupancy_m<4>(ndim, nw, adj);
    case 8: return occupancy_m<8>(ndim, nw, adj);
    default: return 0;
    }
}

void launch_step(int ndim, int M, int nw, bool adj, const Job *jobs, const int *prefix,
                 int njobs, int step, int ttiles, int gblocks, int remap, const LevelMap &lm,
                 hipStream_t st)
{
    switch (M) {
    case 1: launch_step_m<1>(ndim, nw, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, lm, st); break;
    case 2: launch_step_m<2>(ndim, nw, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, lm, st); break;
    case 4: launch_step_m<4>(ndim, nw, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, lm, st); break;
    case 8: launch_step_m<8>(ndim, nw, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, lm, st); break;
    default: break;
    }
}

static int grid_for(int64_t n, int threads, int cap)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

void launch_prep_kappa(const float *v, float *kappa, int M, int gy, int nz, int ny, int nx,
                       int pitch, int nya, int nb, int nzm, int nym, int nxm, int64_t total,
                       float dt_dx, hipStream_t st)
{
    hipLaunchKernelGGL(k_prep_kappa, dim3(grid_for(total, 256, 65536)), dim3(256), 0, st, v,
                       kappa, M, gy, nz, ny, nx, pitch, nya, nb, nzm, nym, nxm, total, dt_dx);
}

// Zero the frame and row padding of nf consecutive fields (fstride floats
// each: nzp planes of nya rows of pitch floats; grid cells are planes
// M .. M+nz-1, rows gy .. gy+ny-1, columns M .. M+nx-1).  One wavefront per
// row: frame rows are cleared whole, grid rows outside columns M .. M+nx-1.
__global__ __launch_bounds__(256) void k_zero_frames(float *__restrict__ f, int64_t nrows,
                                                     int64_t fstride, int nya, int pitch, int M,
                                                     int gy, int nz, int ny, int nx)
{
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int planes = (int)(fstride / ((int64_t)nya * pitch));
    for (int64_t r = w0; r < nrows; r += nw) {
        const int64_t fld = r / ((int64_t)planes * nya);
        const int rem = (int)(r - fld * planes * nya);
        const int z = rem / nya, y = rem - (rem / nya) * nya;
        float *row = f + fld * fstride + ((int64_t)z * nya + y) * pitch;
        const bool frame = z < M || z >= nz + M || y < gy || y >= ny + gy;
        if (frame) {
            float4 *row4 = reinterpret_cast<float4 *>(row);
            for (int c = lane; c < pitch / 4; c += 64) row4[c] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            if (lane < M) row[lane] = 0.f;
            for (int c = nx + M + lane; c < pitch; c += 64) row[c] = 0.f;
        }
    }
}

void launch_zero_frames(float *p, int64_t nfields, int64_t fstride, int nya, int pitch, int M,
                        int gy, int nz, int ny, int nx, hipStream_t st)
{
    const int64_t nrows = nfields * (fstride / pitch);
    hipLaunchKernelGGL(k_zero_frames, dim3(grid_for(nrows * 64, 256, 8192)), dim3(256), 0, st, p,
                       nrows, fstride, nya, pitch, M, gy, nz, ny, nx);
}

void launch_fill(float *p, int64_t n, float val, hipStream_t st)
{
    // n is a multiple of 4 (fields are multiples of 64 floats)
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n / 4, 256, 65536)), dim3(256), 0, st,
                       reinterpret_cast<float4 *>(p), n / 4, val);
}

void launch_snapshot(const Job *jobs, int njobs, int64_t fstride, int slot, int time, int dir,
                     int mask, const LevelMap &lm, hipStream_t st)
{
    hipLaunchKernelGGL(k_snapshot, dim3(grid_for(fstride / 4, 256, 4096), 2 * njobs), dim3(256),
                       0, st, jobs, slot, time, dir, mask, lm);
}

// Multi-step 2-D forward launches: the largest step count per launch, the
// output tile, and the launch itself (M <= 4).
int multi2d_steps() { return 4; }
void multi2d_tile(int M, int *ox, int *oz)
{
    switch (M) {
    case 1: *ox = Multi2d<1, 4>::OX; break;
    case 2: *ox = Multi2d<2, 4>::OX; break;
    default: *ox = Multi2d<4, 4>::OX; break;
    }
    *oz = Multi2d<4, 4>::OZ;
}
void launch_step2d_multi(int M, const Job *jobs, int njobs, int tiles_per_job, int ntxm,
                         int step, int kk, bool record, hipStream_t st)
{
    // 1024 threads: three cells of the 64 x 48 region per thread and step, so
    // a step is a short latency chain (256 threads: 5.3 us per step)
    const dim3 g(njobs * tiles_per_job), b(1024);
    const int rec = record ? 1 : 0;
    switch (M) {
    case 1: hipLaunchKernelGGL((k_step2d_multi<1, 4>), g, b, 0, st, jobs, tiles_per_job, ntxm, step, kk, rec); break;
    case 2: hipLaunchKernelGGL((k_step2d_multi<2, 4>), g, b, 0, st, jobs, tiles_per_job, ntxm, step, kk, rec); break;
    case 4: hipLaunchKernelGGL((k_step2d_multi<4, 4>), g, b, 0, st, jobs, tiles_per_job, ntxm, step, kk, rec); break;
    default: break;
    }
}

void launch_gather(const Job *jobs, const int *gprefix, int njobs, int gblocks, int threads,
                   int step, const LevelMap &lm, hipStream_t st)
{
    if (gblocks > 0)
        hipLaunchKernelGGL(k_gather, dim3(gblocks), dim3(threads), 0, st, jobs, gprefix, njobs,
                           step, lm);
}

void launch_adj_inject(const Job *jobs, const int *gprefix, int njobs, int gblocks, int threads,
                       int step, hipStream_t st)
{
    if (gblocks > 0)
        hipLaunchKernelGGL(k_adj_inject, dim3(gblocks), dim3(threads), 0, st, jobs, gprefix,
                           njobs, step);
}

int misfit_partials() { return 1024; }

void launch_misfit(const float *d, const float *obs, float *res, int64_t n, double *partial,
                   double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_misfit, dim3(misfit_partials()), dim3(256), 0, st, d, obs, res, n,
                       partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, st, partial, misfit_partials(),
                       out);
}

void launch_fold(int ndim, const Job *jobs, int njobs, int M, int gy, int nz, int ny, int nx,
                 int nb, int nzm, int nym, int nxm, float *tmp1, float *tmp2, const float *v,
                 float *dv, hipStream_t st)
{
    (void)nx;
    const int64_t n1 = (int64_t)nz * ny * nxm;
    hipLaunchKernelGGL(k_fold_x, dim3(grid_for(n1, 256, 65536)), dim3(256), 0, st, jobs, njobs,
                       M, gy, nxm, tmp1);
    const float *zin = tmp1;
    if (ndim == 3) {
        const int64_t n2 = (int64_t)nz * nym * nxm;
        hipLaunchKernelGGL(k_fold_y, dim3(grid_for(n2, 256, 65536)), dim3(256), 0, st, tmp1, nz,
                           ny, nym, nxm, nb, tmp2);
        zin = tmp2;
    }
    const int64_t n3 = (int64_t)nzm * nym * nxm;
    hipLaunchKernelGGL(k_fold_z, dim3(grid_for(n3, 256, 65536)), dim3(256), 0, st, zin, v, nz,
                       nzm, nym, nxm, nb, dv);
}

}  // namespace fwi
