// fwi_kernels.hip -- gfx950 kernels of the acoustic FWI hot path.
//
// One launch of a step kernel advances every job of a job table by one time
// step (Eq. 3 of the paper with a sponge; star Laplacian of Fig. 3):
//     out = alpha * (2 p + kappa' * L'p + src) - beta * p_prev
// with L'p = sum_m c_m [(p_{+m} - p) + (p_{-m} - p)] summed over the axes
// (the Laplacian times dx^2, in difference form for fp32 accuracy) and
// kappa' = (v dt / dx)^2.  The adjoint launch applies the same operator to
// the scaled adjoint field psi' (psi = kappa*alpha*lambda, divided by dx^2),
// for which the discrete adjoint recurrence IS the forward recurrence, and
// accumulates the imaging condition g += psi'^{k+1} * L'p^k.
//
// Design for CDNA4 (the paper's MXU band-matrix formulation does not apply:
// the star stencil is banded, not a dense contraction, and the step is HBM
// bound at 16 algorithmic bytes per cell-update):
//  * 3-D: 256-thread blocks own a 64 (x) x 16 (y) column of the grid over a
//    chunk of z planes.  Each thread keeps a register queue of 2M+1 planes
//    for the z-derivative (z marching), the current xy plane with its M-cell
//    halo is staged in LDS for the x and y derivatives, and each thread owns
//    4 consecutive y rows so y-neighbours are reused from LDS.
//  * 2-D: one wavefront per block, 64 columns marching down a chunk of rows.
//  * Each wavefront reads and writes whole aligned 256-byte row segments.
//  * Blocks are remapped so that each XCD (one L2 each) gets a contiguous
//    range of tiles: neighbouring tiles share their halos in the same L2.
//  * Receiver sampling of level n is done by extra blocks of the launch that
//    computes level n+1 (level n is read-only there), so it costs no launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

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
    __host__ __device__ constexpr Weights() : c()
    {
        for (int m = 1; m <= M; ++m) c[m] = float(weightd(M, m));
    }
};

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

// Receiver sampling: traces[n-1][r] = p^n[rec_r] (level n is read-only here).
__device__ __forceinline__ void gather_block(const Job *__restrict__ J, int r, int n)
{
    if (!J->record || n < 1 || n > J->nt || r >= J->nrec) return;
    const float *cur = J->ring + (int64_t)mod_pos(n, J->R) * J->fstride;
    J->traces[(int64_t)(n - 1) * J->nrec + r] = cur[J->rec_off[r]];
}

// --------------------------------------------------------------- 3-D step
template <int M, bool ADJ>
__global__ __launch_bounds__(256) void k_step3d(const Job *__restrict__ jobs,
                                                const int *__restrict__ prefix, int njobs,
                                                int step, int ttiles, int remap)
{
    constexpr int TX = kTileX, RY = kRowsPerWave, TY = kTileY;
    constexpr int LX = TX + 2 * M, LY = TY + 2 * M, Q = 2 * M + 1;
    constexpr Weights<M> W{};
    __shared__ float sp[LY * LX];
    __shared__ float sf[ADJ ? LY * LX : 1];

    const int tid = threadIdx.x;
    int b = blockIdx.x;
    if (b >= ttiles) {   // receiver-sampling blocks (forward launches only)
        if constexpr (ADJ) return;
        const int gb = b - ttiles;
        const int j = find_job(prefix + njobs + 1, njobs, gb);
        const Job *J = jobs + j;
        gather_block(J, (gb - prefix[njobs + 1 + j]) * blockDim.x + tid, J->n0 + step);
        return;
    }
    if (remap) b = xcd_remap(b, ttiles);
    const int j = find_job(prefix, njobs, b);
    const Job *__restrict__ J = jobs + j;
    const int n = ADJ ? J->k0 - step : J->n0 + step;
    if (ADJ ? (n < 1 || n > J->nt) : (n < 0 || n >= J->nt)) return;

    const int nz = J->nz, ny = J->ny, nx = J->nx, pitch = J->pitch, nb = J->nb;
    const int64_t plane = J->plane, fstride = J->fstride;
    int local = b - prefix[j];
    const int tx = local % J->ntx;
    local /= J->ntx;
    const int ty = local % J->nty;
    const int tz = local / J->nty;
    const int z0 = tz * J->zc, z1 = min(z0 + J->zc, nz);

    // field levels: forward p^n -> p^{n+1}; adjoint psi^{k+1} -> psi^k
    const float *cur, *prv;
    float *out;
    const float *fwd = nullptr;
    float *grad = nullptr;
    bool accum = false;
    if (ADJ) {
        cur = J->adj + (int64_t)((n + 1) & 1) * fstride;
        prv = J->adj + (int64_t)(n & 1) * fstride;
        out = J->adj + (int64_t)(n & 1) * fstride;
        accum = J->accumulate && n <= J->nt - 1;
        fwd = J->ring + (int64_t)mod_pos(n, J->R) * fstride;
        grad = J->grad;
    } else {
        cur = J->ring + (int64_t)mod_pos(n, J->R) * fstride;
        prv = J->ring + (int64_t)mod_pos(n - 1, J->R) * fstride;
        out = J->ring + (int64_t)mod_pos(n + 1, J->R) * fstride;
    }
    const float *kap = J->kappa;
    const float eta_dt = J->eta_dt;

    const int lane = tid & 63, wv = tid >> 6;
    const int col = tx * TX + lane;   // memory column
    const int x = col - M;            // padded-grid x
    const bool ax = x >= 0 && x < nx;
    int yy[RY];
    bool act[RY];
    int64_t roff[RY];
    int dy2[RY];
    const int dxs = sponge_depth(x, nx, nb);
#pragma unroll
    for (int i = 0; i < RY; ++i) {
        yy[i] = ty * TY + wv * RY + i;
        act[i] = ax && yy[i] < ny;
        roff[i] = (int64_t)(yy[i] + M) * pitch + col;
        const int d = sponge_depth(yy[i], ny, nb);
        dy2[i] = d * d + dxs * dxs;
    }
    float srcv = 0.f;
    int src_lrow = -1;
    if (!ADJ && J->src_z >= z0 && J->src_z < z1 && J->src_x == x) {
        const int r = J->src_y - (ty * TY + wv * RY);
        if (r >= 0 && r < RY) { src_lrow = r; srcv = J->src_scale * J->wavelet[n]; }
    }

    float q[RY][Q];
    float f[ADJ ? RY : 1][ADJ ? Q : 1];
#pragma unroll
    for (int s = 0; s < 2 * M; ++s) {
        const int64_t po = (int64_t)(z0 + s) * plane;   // plane z0 - M + s
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            q[i][s] = act[i] ? cur[po + roff[i]] : 0.f;
            if constexpr (ADJ) f[i][s] = act[i] ? fwd[po + roff[i]] : 0.f;
        }
    }

    for (int z = z0; z < z1; ++z) {
        const int64_t pz = (int64_t)(z + M) * plane;   // plane z
        const int64_t pf = pz + (int64_t)M * plane;    // plane z + M
        float kv[RY], pv[RY];
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            q[i][2 * M] = act[i] ? cur[pf + roff[i]] : 0.f;
            if constexpr (ADJ) f[i][2 * M] = act[i] ? fwd[pf + roff[i]] : 0.f;
            kv[i] = act[i] ? kap[pz + roff[i]] : 0.f;
            pv[i] = act[i] ? prv[pz + roff[i]] : 0.f;
        }
        // stage plane z with its halo in LDS
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            sp[(M + wv * RY + i) * LX + M + lane] = q[i][M];
            if constexpr (ADJ) sf[(M + wv * RY + i) * LX + M + lane] = f[i][M];
        }
        for (int h = tid; h < 2 * M * TX; h += 256) {   // rows above and below
            const int r = h / TX, c = h % TX;
            const int ly = r < M ? r : r + TY;
            const int yg = ty * TY - M + ly;
            float a = 0.f, bq = 0.f;
            if (yg < ny + M) {
                const int64_t o = pz + (int64_t)(yg + M) * pitch + tx * TX + c;
                a = cur[o];
                if constexpr (ADJ) bq = fwd[o];
            }
            sp[ly * LX + M + c] = a;
            if constexpr (ADJ) sf[ly * LX + M + c] = bq;
        }
        for (int h = tid; h < TY * 2 * M; h += 256) {   // columns left and right
            const int r = h / (2 * M), c = h % (2 * M);
            const int lc = c < M ? c : c + TX;
            const int cm = tx * TX - M + lc;
            const int yg = ty * TY + r;
            float a = 0.f, bq = 0.f;
            if (cm >= 0 && cm < pitch && yg < ny + M) {
                const int64_t o = pz + (int64_t)(yg + M) * pitch + cm;
                a = cur[o];
                if constexpr (ADJ) bq = fwd[o];
            }
            sp[(M + r) * LX + lc] = a;
            if constexpr (ADJ) sf[(M + r) * LX + lc] = bq;
        }
        __syncthreads();

        const int dz = sponge_depth(z, nz, nb);
#pragma unroll
        for (int i = 0; i < RY; ++i) {
            if (!act[i]) continue;
            const int ly = M + wv * RY + i, lx = M + lane;
            const float pc = q[i][M];
            float acc = 0.f;
#pragma unroll
            for (int m = M; m >= 1; --m) {
                const float d = ((sp[ly * LX + lx + m] - pc) + (sp[ly * LX + lx - m] - pc)) +
                                ((sp[(ly + m) * LX + lx] - pc) + (sp[(ly - m) * LX + lx] - pc)) +
                                ((q[i][M + m] - pc) + (q[i][M - m] - pc));
                acc = fmaf(W.c[m], d, acc);
            }
            float val = fmaf(kv[i], acc, 2.f * pc);
            if (!ADJ && i == src_lrow && z == J->src_z) val += srcv;
            const int d2 = dy2[i] + dz * dz;
            float o;
            if (d2 == 0) {
                o = val - pv[i];
            } else {
                const float e = eta_dt * (float)d2;
                const float a = 1.f / (1.f + e);
                o = a * val - (1.f - e) * a * pv[i];
            }
            out[pz + roff[i]] = o;
            if constexpr (ADJ) if (accum) {
                const float fc = f[i][M];
                float lf = 0.f;
#pragma unroll
                for (int m = M; m >= 1; --m) {
                    const float d = ((sf[ly * LX + lx + m] - fc) + (sf[ly * LX + lx - m] - fc)) +
                                    ((sf[(ly + m) * LX + lx] - fc) + (sf[(ly - m) * LX + lx] - fc)) +
                                    ((f[i][M + m] - fc) + (f[i][M - m] - fc));
                    lf = fmaf(W.c[m], d, lf);
                }
                grad[pz + roff[i]] += pc * lf;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2 * M; ++s) {
#pragma unroll
            for (int i = 0; i < RY; ++i) {
                q[i][s] = q[i][s + 1];
                if constexpr (ADJ) f[i][s] = f[i][s + 1];
            }
        }
    }
}

// --------------------------------------------------------------- 2-D step
template <int M, bool ADJ>
__global__ __launch_bounds__(64) void k_step2d(const Job *__restrict__ jobs,
                                               const int *__restrict__ prefix, int njobs,
                                               int step, int ttiles, int remap)
{
    constexpr int TX = kTileX, LX = TX + 2 * M, Q = 2 * M + 1;
    constexpr Weights<M> W{};
    __shared__ float sp[LX];
    __shared__ float sf[ADJ ? LX : 1];

    const int lane = threadIdx.x;
    int b = blockIdx.x;
    if (b >= ttiles) {
        if constexpr (ADJ) return;
        const int gb = b - ttiles;
        const int j = find_job(prefix + njobs + 1, njobs, gb);
        const Job *J = jobs + j;
        gather_block(J, (gb - prefix[njobs + 1 + j]) * blockDim.x + lane, J->n0 + step);
        return;
    }
    if (remap) b = xcd_remap(b, ttiles);
    const int j = find_job(prefix, njobs, b);
    const Job *__restrict__ J = jobs + j;
    const int n = ADJ ? J->k0 - step : J->n0 + step;
    if (ADJ ? (n < 1 || n > J->nt) : (n < 0 || n >= J->nt)) return;

    const int nz = J->nz, nx = J->nx, pitch = J->pitch, nb = J->nb;
    const int64_t fstride = J->fstride;
    int local = b - prefix[j];
    const int tx = local % J->ntx;
    const int tz = local / J->ntx;
    const int z0 = tz * J->zc, z1 = min(z0 + J->zc, nz);

    const float *cur, *prv;
    float *out;
    const float *fwd = nullptr;
    float *grad = nullptr;
    bool accum = false;
    if (ADJ) {
        cur = J->adj + (int64_t)((n + 1) & 1) * fstride;
        prv = J->adj + (int64_t)(n & 1) * fstride;
        out = J->adj + (int64_t)(n & 1) * fstride;
        accum = J->accumulate && n <= J->nt - 1;
        fwd = J->ring + (int64_t)mod_pos(n, J->R) * fstride;
        grad = J->grad;
    } else {
        cur = J->ring + (int64_t)mod_pos(n, J->R) * fstride;
        prv = J->ring + (int64_t)mod_pos(n - 1, J->R) * fstride;
        out = J->ring + (int64_t)mod_pos(n + 1, J->R) * fstride;
    }
    const float *kap = J->kappa;
    const float eta_dt = J->eta_dt;

    const int col = tx * TX + lane;
    const int x = col - M;
    const bool act = x >= 0 && x < nx;
    const int dxs = sponge_depth(x, nx, nb);
    float srcv = 0.f;
    const bool src_here = !ADJ && J->src_x == x && J->src_z >= z0 && J->src_z < z1;
    if (src_here) srcv = J->src_scale * J->wavelet[n];

    float q[Q];
    float f[ADJ ? Q : 1];
#pragma unroll
    for (int s = 0; s < 2 * M; ++s) {
        const int64_t o = (int64_t)(z0 + s) * pitch + col;   // row z0 - M + s
        q[s] = act ? cur[o] : 0.f;
        if constexpr (ADJ) f[s] = act ? fwd[o] : 0.f;
    }
    for (int z = z0; z < z1; ++z) {
        const int64_t oz = (int64_t)(z + M) * pitch + col;
        const int64_t of = oz + (int64_t)M * pitch;
        q[2 * M] = act ? cur[of] : 0.f;
        if constexpr (ADJ) f[2 * M] = act ? fwd[of] : 0.f;
        const float kv = act ? kap[oz] : 0.f;
        const float pv = act ? prv[oz] : 0.f;
        sp[M + lane] = q[M];
        if constexpr (ADJ) sf[M + lane] = f[M];
        if (lane < 2 * M) {
            const int lc = lane < M ? lane : lane + TX;
            const int cm = tx * TX - M + lc;
            float a = 0.f, bq = 0.f;
            if (cm >= 0 && cm < pitch) {
                const int64_t o = (int64_t)(z + M) * pitch + cm;
                a = cur[o];
                if constexpr (ADJ) bq = fwd[o];
            }
            sp[lc] = a;
            if constexpr (ADJ) sf[lc] = bq;
        }
        __syncthreads();
        if (act) {
            const int lx = M + lane;
            const float pc = q[M];
            float acc = 0.f;
#pragma unroll
            for (int m = M; m >= 1; --m) {
                const float d = ((sp[lx + m] - pc) + (sp[lx - m] - pc)) +
                                ((q[M + m] - pc) + (q[M - m] - pc));
                acc = fmaf(W.c[m], d, acc);
            }
            float val = fmaf(kv, acc, 2.f * pc);
            if (!ADJ && src_here && z == J->src_z) val += srcv;
            const int dz = sponge_depth(z, nz, nb);
            const int d2 = dxs * dxs + dz * dz;
            float o;
            if (d2 == 0) {
                o = val - pv;
            } else {
                const float e = eta_dt * (float)d2;
                const float a = 1.f / (1.f + e);
                o = a * val - (1.f - e) * a * pv;
            }
            out[oz] = o;
            if constexpr (ADJ) if (accum) {
                const float fc = f[M];
                float lf = 0.f;
#pragma unroll
                for (int m = M; m >= 1; --m) {
                    const float d = ((sf[lx + m] - fc) + (sf[lx - m] - fc)) +
                                    ((f[M + m] - fc) + (f[M - m] - fc));
                    lf = fmaf(W.c[m], d, lf);
                }
                grad[oz] += pc * lf;
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2 * M; ++s) {
            q[s] = q[s + 1];
            if constexpr (ADJ) f[s] = f[s + 1];
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
// dir 0: ring -> snap[slot]; 1: snap[slot] -> ring; 2: zero the two levels (t = 0).
__global__ void k_snapshot(const Job *__restrict__ jobs, int slot, int time, int dir)
{
    const Job *J = jobs + (blockIdx.y >> 1);
    const int which = blockIdx.y & 1;
    float4 *r = reinterpret_cast<float4 *>(J->ring + (int64_t)mod_pos(time - which, J->R) * J->fstride);
    float4 *s = reinterpret_cast<float4 *>(J->snap + (int64_t)(2 * slot + which) * J->fstride);
    const int64_t n4 = J->fstride / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (dir == 0) s[i] = r[i];
        else if (dir == 1) r[i] = s[i];
        else r[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Final receiver sampling (level n = n0 + step).
__global__ void k_gather(const Job *__restrict__ jobs, const int *__restrict__ gprefix,
                         int njobs, int step)
{
    const int j = find_job(gprefix, njobs, blockIdx.x);
    const Job *J = jobs + j;
    gather_block(J, (blockIdx.x - gprefix[j]) * blockDim.x + threadIdx.x, J->n0 + step);
}

// Adjoint source: psi'^k[rec] += kappa'[rec] * res[k-1][rec] (alpha = 1 on the
// model grid, where every receiver sits).  Receivers sharing a cell are summed
// by the first of them, in index order, so the result is deterministic.
__global__ void k_adj_inject(const Job *__restrict__ jobs, const int *__restrict__ gprefix,
                             int njobs, int step)
{
    const int j = find_job(gprefix, njobs, blockIdx.x);
    const Job *J = jobs + j;
    const int k = J->k0 - step;
    const int r = (blockIdx.x - gprefix[j]) * blockDim.x + threadIdx.x;
    if (k < 1 || k > J->nt || r >= J->nrec || !J->rec_head[r]) return;
    const float *res = J->res + (int64_t)(k - 1) * J->nrec;
    float s = res[r];
    for (int q = J->rec_next[r]; q >= 0; q = J->rec_next[q]) s += res[q];
    const int64_t off = J->rec_off[r];
    float *psi = J->adj + (int64_t)(k & 1) * J->fstride;
    psi[off] += J->kappa[off] * s;
}

// Misfit (Eq. 1) and adjoint source: res = 2 (d - obs); per-block partial sums
// of (d - obs)^2 in fp64, reduced in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_misfit(const float *__restrict__ d,
                                                const float *__restrict__ obs,
                                                float *__restrict__ res, int64_t n,
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

// ---------------------------------------------------------------- launchers
int vstats_blocks() { return 256; }

void launch_vstats(const float *v, int64_t n, float *partial, hipStream_t st)
{
    hipLaunchKernelGGL(k_vstats, dim3(vstats_blocks()), dim3(256), 0, st, v, n, partial);
}

template <int M>
static void launch_step_m(int ndim, bool adj, const Job *jobs, const int *prefix, int njobs,
                          int step, int ttiles, int gblocks, int remap, hipStream_t st)
{
    const int grid = ttiles + (adj ? 0 : gblocks);
    if (grid <= 0) return;
    if (ndim == 3) {
        if (adj)
            hipLaunchKernelGGL((k_step3d<M, true>), dim3(grid), dim3(256), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap);
        else
            hipLaunchKernelGGL((k_step3d<M, false>), dim3(grid), dim3(256), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap);
    } else {
        if (adj)
            hipLaunchKernelGGL((k_step2d<M, true>), dim3(grid), dim3(64), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap);
        else
            hipLaunchKernelGGL((k_step2d<M, false>), dim3(grid), dim3(64), 0, st, jobs, prefix,
                               njobs, step, ttiles, remap);
    }
}

void launch_step(int ndim, int M, bool adj, const Job *jobs, const int *prefix, int njobs,
                 int step, int ttiles, int gblocks, int remap, hipStream_t st)
{
    switch (M) {
    case 1: launch_step_m<1>(ndim, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, st); break;
    case 2: launch_step_m<2>(ndim, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, st); break;
    case 4: launch_step_m<4>(ndim, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, st); break;
    case 8: launch_step_m<8>(ndim, adj, jobs, prefix, njobs, step, ttiles, gblocks, remap, st); break;
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

void launch_fill(float *p, int64_t n, float val, hipStream_t st)
{
    // n is a multiple of 4 (fields are multiples of 64 floats)
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n / 4, 256, 65536)), dim3(256), 0, st,
                       reinterpret_cast<float4 *>(p), n / 4, val);
}

void launch_snapshot(const Job *jobs, int njobs, int64_t fstride, int slot, int time, int dir,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_snapshot, dim3(grid_for(fstride / 4, 256, 4096), 2 * njobs), dim3(256),
                       0, st, jobs, slot, time, dir);
}

void launch_gather(const Job *jobs, const int *gprefix, int njobs, int gblocks, int threads,
                   int step, hipStream_t st)
{
    if (gblocks > 0)
        hipLaunchKernelGGL(k_gather, dim3(gblocks), dim3(threads), 0, st, jobs, gprefix, njobs,
                           step);
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
