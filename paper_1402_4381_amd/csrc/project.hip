// Forward projection (ray-driven Joseph) and the image-layout / x-update
// kernel that feeds it.
//
// Data layout.  The projector never reads the caller's [z][y][x] image.  It
// reads two zero-padded copies that the x-update kernel writes as a side
// product of every update:
//   XT[i][k+2][j+2]  (x-dominant rays: y fastest)   size nx * (nz+4) * (ny+4)
//   XN[j][k+2][i+2]  (y-dominant rays: x fastest)   size ny * (nz+4) * (nx+4)
// (2D: no z padding).  A wavefront holds 64 adjacent detector channels of one
// view and row; at a given slice their interpolation positions are adjacent,
// so each tap load touches a few contiguous cache lines.  The two-voxel zero
// border on every interpolated axis lets the inner loop clamp indices instead
// of testing bounds: a clamped out-of-range tap always reads a zero.
#include "lalm_internal.h"

namespace lalm {
namespace {

struct FPArgs {
    GeoK k;
    const RayRec *rays;     // subset's rays, [view][bin]
    const RayRecZ *raysz;   // 3D
    const ViewRec *views;   // subset's views
    const float *rowv, *rowf;
    const float *XT, *XN;
    long long nrays;
    const float *y, *w;
    float *out;
    double *partials;       // mode 1
    const DevScalars *st_sc;   // skip when its status is set (LALM steps only)
    // DEC: the pending continuation decision, then the selected layouts
    const float *XT1, *XN1;
    const DevScalars *sc_in;
    DevScalars *sc_out;
    const double *dec_part;
    long long dec_n;
    ContArgs cont;
    int ray_scaled;         // 3D mode 0: out also carries the ray's scale
    // batch: image b = blockIdx.y; its y and w start b s_yw further, its
    // output b s_out further
    BatchStr bs;
    long long s_yw, s_out;
};

constexpr int FP3_U = 8;   // 3D: samples whose taps are loaded together
constexpr int FP2_U = 8;   // 2D: samples per round of the main loop (12, 16 and 24 measured slower)

// U consecutive samples s..s+U-1 of a 2D ray: their tap pairs are loaded
// before any is used, and the interpolated values are added in sample order.
// rowp points at slice row s of the layout; in-round offsets stay 32-bit.
template <int U>
__device__ __forceinline__ void fp2d_round(float &acc, int s, const float *rowp, const RayRec &rr,
                                           int ld, int lim)
{
    float v0[U], v1[U], f[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float eta = fmaf((float)(s + u), rr.c, rr.a);
        const float fl = floorf(eta);
        f[u] = eta - fl;
        const int j0 = min(max((int)fl, -2), lim);
        const float *pp = rowp + (u * ld + j0);
        v0[u] = pp[0];
        v1[u] = pp[1];
    }
    // keep the scheduler from interleaving the loads with the sums below
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) acc += fmaf(f[u], v1[u] - v0[u], v0[u]);
}

template <bool IS3D, int NSEG, int MODE, bool DEC>
__global__ void __launch_bounds__(64 * NSEG) fp_kernel(FPArgs A)
{
    const GeoK &K = A.k;
    const int lane = threadIdx.x, seg = threadIdx.y;
    {
        // image bi of the batch
        const long long bi = blockIdx.y;
        A.XT += bi * A.bs.layT;
        A.XN += bi * A.bs.layN;
        if (A.XT1) A.XT1 += bi * A.bs.layT;
        if (A.XN1) A.XN1 += bi * A.bs.layN;
        if (A.y) A.y += bi * A.s_yw;
        if (A.w) A.w += bi * A.s_yw;
        if (A.out) A.out += bi * A.s_out;
        if (A.partials) A.partials += bi * A.bs.part;
        if (A.st_sc) A.st_sc += bi;
        if (A.sc_in) A.sc_in += bi;
        if (A.sc_out) A.sc_out += bi;
        if (A.dec_part) A.dec_part += bi * A.bs.part;
        A.cont = cont_at(A.cont, (int)bi);
    }
    const long long q = (long long)blockIdx.x * 64 + lane;
    const bool valid = q < A.nrays;
    float acc = 0.0f;
    RayRec rr{0.f, 0.f, 0.f, 1u};
    int r = 0, kv = 0, b = 0;
    float yv = 0.0f, wv = 1.0f;
    // loads that do not depend on the image go out first
    if (valid) {
        b = (int)(q % K.nb);
        const long long vrow = q / K.nb;
        r = IS3D ? (int)(vrow % K.nr) : 0;
        kv = IS3D ? (int)(vrow / K.nr) : (int)vrow;
        rr = A.rays[(long long)kv * K.nb + b];
        if (seg == 0) {
            if (A.y) yv = A.y[q];
            if (A.w) wv = A.w[q];
        }
    }
    const float *XT = A.XT, *XN = A.XN;
    if (DEC) {
        // every wave reduces the same partials in the same order, so all
        // take the same decision; one thread records it
        const double xi = fixed_sum_wave(A.dec_part, A.dec_n, lane);
        const DevScalars s0 = *A.sc_in;
        const bool lead = blockIdx.x == 0 && lane == 0 && seg == 0;
        if (s0.status) {
            if (lead) *A.sc_out = s0;
            return;
        }
        const DevScalars s1 = continuation_update(s0, A.cont, xi, false, lead);
        if (lead) *A.sc_out = s1;
        if (s1.status) return;
        if (s1.sel) {
            XT = A.XT1;
            XN = A.XN1;
        }
    } else if (A.st_sc && A.st_sc->status) {
        return;
    }
    if (valid) {
        const bool ydom = meta_ydom(rr.meta);
        const int ns = ydom ? K.ny : K.nx;
        const int seglen = (ns + NSEG - 1) / NSEG;
        int s0 = max(meta_lo(rr.meta), seg * seglen);
        int s1 = min(meta_hi(rr.meta), seg * seglen + seglen - 1);
        const float *img = ydom ? XN : XT;
        const int lim = ydom ? K.nx : K.ny;
        if (!IS3D) {
            const int ld = ydom ? K.ldN : K.ldT;
            int s = s0;
            // the slice row of sample s; in-round offsets are 32-bit
            const float *rowp = img + 2 + (long long)s0 * ld;
            // FP2_U samples per round, then 4: the tap loads of a round are
            // independent and go out together
            for (; s + FP2_U - 1 <= s1; s += FP2_U, rowp += FP2_U * ld)
                fp2d_round<FP2_U>(acc, s, rowp, rr, ld, lim);
            if (s + 3 <= s1) {
                fp2d_round<4>(acc, s, rowp, rr, ld, lim);
                s += 4;
                rowp += 4 * ld;
            }
            for (; s <= s1; ++s, rowp += ld) {
                const float eta = fmaf((float)s, rr.c, rr.a);
                const float fl = floorf(eta);
                const float f = eta - fl;
                const int j0 = min(max((int)fl, -2), lim);
                const float *pp = rowp + j0;
                const float v0 = pp[0], v1 = pp[1];
                acc += fmaf(f, v1 - v0, v0);
            }
        } else {
            const RayRecZ rz = A.raysz[(long long)kv * K.nb + b];
            const float z0 = A.views[kv].z0;
            const float vr = A.rowv[r];
            // restrict to the slices where zeta = z0 + vr*(m + s*k) lies in
            // [-1, nz); one slice of margin covers FP32 rounding
            const float slope = vr * rz.k, off = fmaf(vr, rz.m, z0);
            if (slope != 0.0f) {
                float ta = (-1.0f - off) / slope, tb = ((float)K.nz - off) / slope;
                float lo = fminf(ta, tb), hi = fmaxf(ta, tb);
                lo = fmaxf(lo, -4.0f);
                hi = fminf(hi, (float)(ns + 4));
                s0 = max(s0, (int)floorf(lo) - 1);
                s1 = min(s1, (int)ceilf(hi) + 1);
            } else if (!(off >= -1.0f && off < (float)K.nz)) {
                s1 = s0 - 1;
            }
            const int ld = ydom ? K.ldN : K.ldT;
            const long long slab = ydom ? K.slabN : K.slabT;
            const float *base = img + 2 * ld + 2;
            // FP3_U samples per round: their tap loads go out together
            int s = s0;
            for (; s + FP3_U - 1 <= s1; s += FP3_U) {
                float v00[FP3_U], v01[FP3_U], v10[FP3_U], v11[FP3_U], f[FP3_U], h[FP3_U];
#pragma unroll
                for (int u = 0; u < FP3_U; ++u) {
                    const float eta = fmaf((float)(s + u), rr.c, rr.a);
                    const float qz = fmaf((float)(s + u), rz.k, rz.m);
                    const float zeta = fmaf(vr, qz, z0);
                    const float fl = floorf(eta), zl = floorf(zeta);
                    f[u] = eta - fl;
                    h[u] = zeta - zl;
                    const int j0 = min(max((int)fl, -2), lim);
                    const int k0 = min(max((int)zl, -2), K.nz);
                    const float *pp = base + (long long)(s + u) * slab + (long long)k0 * ld + j0;
                    v00[u] = pp[0]; v01[u] = pp[1]; v10[u] = pp[ld]; v11[u] = pp[ld + 1];
                }
#pragma unroll
                for (int u = 0; u < FP3_U; ++u) {
                    const float lo = fmaf(f[u], v01[u] - v00[u], v00[u]);
                    const float up = fmaf(f[u], v11[u] - v10[u], v10[u]);
                    acc += fmaf(h[u], up - lo, lo);
                }
            }
            for (; s <= s1; ++s) {
                const float eta = fmaf((float)s, rr.c, rr.a);
                const float qz = fmaf((float)s, rz.k, rz.m);
                const float zeta = fmaf(vr, qz, z0);
                const float fl = floorf(eta), zl = floorf(zeta);
                const float f = eta - fl, h = zeta - zl;
                const int j0 = min(max((int)fl, -2), lim);
                const int k0 = min(max((int)zl, -2), K.nz);
                const float *pp = base + (long long)s * slab + (long long)k0 * ld + j0;
                const float v00 = pp[0], v01 = pp[1], v10 = pp[ld], v11 = pp[ld + 1];
                const float lo = fmaf(f, v01 - v00, v00);
                const float up = fmaf(f, v11 - v10, v10);
                acc += fmaf(h, up - lo, lo);
            }
        }
    }
    if (NSEG > 1) {
        __shared__ float red[NSEG][64];
        red[seg][lane] = acc;
        __syncthreads();
        if (seg != 0) return;
        acc = red[0][lane];
#pragma unroll
        for (int t = 1; t < NSEG; ++t) acc += red[t][lane];
    }
    float val = 0.0f;
    if (valid) {
        const float rowf = IS3D ? A.rowf[r] : 1.0f;
        const float proj = acc * rr.sc * rowf;
        val = proj - yv;
        if (MODE == 0) A.out[q] = (IS3D && A.ray_scaled) ? wv * val * (rr.sc * rowf) : wv * val;
    }
    if (MODE == 1) {
        // 1/2 w e^2 summed in FP64 over the block's rays (one wavefront)
        double t = valid ? 0.5 * (double)wv * (double)val * (double)val : 0.0;
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) A.partials[blockIdx.x] = t;
    }
}

template <bool IS3D, int NSEG>
hipError_t fp_dispatch_mode(const lalm_plan *p, const FPArgs &a, int mode, long long nblk, hipStream_t st)
{
    dim3 blk(64, NSEG), grd((unsigned)nblk, (unsigned)p->B);
    // mode 2: mode 0 after the pending continuation decision (2D)
    if (mode == 0) return klaunch(p, fp_kernel<IS3D, NSEG, 0, false>, grd, blk, st, a);
    if (mode == 1) return klaunch(p, fp_kernel<IS3D, NSEG, 1, false>, grd, blk, st, a);
    if (!IS3D) return klaunch(p, fp_kernel<false, NSEG, 0, true>, grd, blk, st, a);
    return hipErrorInvalidValue;
}

template <bool IS3D>
hipError_t fp_dispatch(const lalm_plan *p, const FPArgs &a, int nseg, int mode, long long nblk, hipStream_t st)
{
    switch (nseg) {
    case 1: return fp_dispatch_mode<IS3D, 1>(p, a, mode, nblk, st);
    case 2: return fp_dispatch_mode<IS3D, 2>(p, a, mode, nblk, st);
    case 4: return fp_dispatch_mode<IS3D, 4>(p, a, mode, nblk, st);
    default: return fp_dispatch_mode<IS3D, 8>(p, a, mode, nblk, st);
    }
}

// ---------------------------------------------------------------- x-update
//
// One thread per pixel of a 32x32 (x, y) tile, for one z slice (2D and the
// first of several inner iterations) or UPD_ZS consecutive slices (3D
// launches that store the padded layouts).  Writes the caller's image
// (UPD_STEP), XN directly (x fastest) and XT through an LDS transpose (y
// fastest), so every global store is coalesced.
constexpr int UPD_ZS = 2;
struct UpdArgs {
    GeoK k;
    float *x;
    const float *G, *g, *gradR, *denom;
    float *XT, *XN;
    const DevScalars *sc;   // scalars of this step (or of the previous one, do_finalize)
    float beta;
    int nonneg;
    // fused continuation decision of the previous step (UPD_STEP)
    int do_finalize;
    const double *partials;
    long long nblocks;
    DevScalars *sc_out;
    ContArgs cont;
    // first of several inner iterations: v and the next momentum point go here
    float *vout, *zout;
    BatchStr bs;            // image b of the batch: tiles of slice groups b nzb ..
    int nimg;               // images in the batch
};

template <bool IS3D, int MODE, int ZS>
__global__ void __launch_bounds__(1024, 8) update_kernel(UpdArgs A)
{
    // a thread takes ZS consecutive slices of its (x, y) pixel and issues the
    // loads of all of them before any arithmetic, so a wave keeps ZS times
    // the bytes of one voxel's five loads in flight
    const GeoK &K = A.k;
    __shared__ float tile[ZS][32][33];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const unsigned nzb = (unsigned)(K.nz + ZS - 1) / ZS;      // slice groups per image
    // tile of this block, in (x, y, slice group, image) order.  A launch
    // that stores the padded layouts: the hardware hands consecutive blocks
    // to the eight XCDs in turn, and XCD c takes the c-th eighth of the
    // tiles, so the tiles beside a tile, whose stores complete the cache
    // lines that its row segments of those layouts begin or end in, mostly
    // store through the same L2.  The first of several inner iterations
    // (vout) stores no layout and keeps the round-robin order, in which the
    // XCDs work on neighbouring tiles and share the Infinity Cache, and one
    // slice per thread (both measured faster there).  The grid is padded to
    // a multiple of 8; padding blocks have no tile.
    const unsigned ntx = (unsigned)(K.nx + 31) / 32, nty = (unsigned)(K.ny + 31) / 32;
    const unsigned tl = A.vout ? blockIdx.x : (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if (tl >= ntx * nty * nzb * A.nimg) return;
    const unsigned bxt = tl % ntx, byt = (tl / ntx) % nty, bzt = tl / (ntx * nty);
    const int k0 = (int)(bzt % nzb) * ZS;
    {
        // image bi of the batch
        const long long bi = bzt / nzb;
        if (A.x) A.x += bi * A.bs.img;
        if (A.G) A.G += bi * A.bs.img;
        if (A.g) A.g += bi * A.bs.img;
        if (A.gradR) A.gradR += bi * A.bs.img;
        if (A.denom) A.denom += bi * A.bs.img;
        A.XT += bi * A.bs.layT;
        A.XN += bi * A.bs.layN;
        A.sc += bi;
        A.sc_out += bi;
        if (A.partials) A.partials += bi * A.bs.part;
        A.cont = cont_at(A.cont, (int)bi);
        if (A.vout) A.vout += bi * A.bs.img;
        if (A.zout) A.zout += bi * A.bs.img;
    }
    const int i = (int)bxt * 32 + tx, j = (int)byt * 32 + ty;
    const long long plane = (long long)K.nx * K.ny;
    const long long idx0 = ((long long)k0 * K.ny + j) * K.nx + i;
    bool in[ZS];
#pragma unroll
    for (int z = 0; z < ZS; ++z) in[z] = i < K.nx && j < K.ny && k0 + z < K.nz;
    // operands first: their loads overlap the continuation decision below
    float v[ZS], Gv[ZS], gv[ZS], rv[ZS], dv[ZS];
#pragma unroll
    for (int z = 0; z < ZS; ++z) {
        v[z] = Gv[z] = gv[z] = rv[z] = dv[z] = 0.0f;
        if (in[z]) {
            const long long idx = idx0 + z * plane;
            if (MODE == UPD_ONES) {
                v[z] = 1.0f;
            } else {
                v[z] = A.x[idx];
                if (MODE == UPD_STEP) {
                    Gv[z] = A.G[idx];
                    gv[z] = A.g[idx];
                    rv[z] = A.gradR[idx];
                    dv[z] = A.denom[idx];
                }
            }
        }
    }
    if (MODE == UPD_STEP) {
        DevScalars s = *A.sc;
        if (A.do_finalize) {
            // every wave takes the same decision from the same fixed-order
            // sum; the first thread records it in the other scalar record
            const bool lead = bxt == 0 && byt == 0 && k0 == 0 && tx == 0 && ty == 0;
            if (!s.status) {
                const double xi = fixed_sum_wave(A.partials, A.nblocks, (tx + 32 * ty) & 63);
                s = continuation_update(s, A.cont, xi, false, lead);
            }
            if (lead) *A.sc_out = s;
        }
        if (s.status) return;
        const float rho = (float)s.rho;
#pragma unroll
        for (int z = 0; z < ZS; ++z) {
            if (!in[z]) continue;
            const long long idx = idx0 + z * plane;
            v[z] = x_update(v[z], Gv[z], gv[z], rv[z], rho, (float)s.alpha, dv[z],
                            A.beta * reg_curv_sum(K, i, j, k0 + z), A.nonneg);
            if (A.vout) {
                A.vout[idx] = v[z];               // first FISTA momentum is zero: z = v
                A.zout[idx] = v[z];
            } else {
                A.x[idx] = v[z];
            }
        }
        if (A.vout) return;                       // the projector layouts follow the last inner iteration
    }
#pragma unroll
    for (int z = 0; z < ZS; ++z) {
        const int k = k0 + z;
        if (in[z]) {
            const long long n_idx = IS3D ? ((long long)j * K.slabN + (long long)(k + 2) * K.ldN + i + 2)
                                         : ((long long)j * K.ldN + i + 2);
            A.XN[n_idx] = v[z];
        }
        tile[z][ty][tx] = v[z];
    }
    __syncthreads();
    {
        const int it = (int)bxt * 32 + ty, jt = (int)byt * 32 + tx;
#pragma unroll
        for (int z = 0; z < ZS; ++z) {
            const int k = k0 + z;
            if (it < K.nx && jt < K.ny && k < K.nz) {
                const long long t_idx = IS3D ? ((long long)it * K.slabT + (long long)(k + 2) * K.ldT + jt + 2)
                                             : ((long long)it * K.ldT + jt + 2);
                A.XT[t_idx] = tile[z][tx][ty];
            }
        }
    }
}

// ---------------------------------------------------------------- inner FISTA
//
// Iteration i >= 2 of the FISTA solve of the step's constrained-denoising
// problem (Sec. IV-A), one thread per voxel of a 32x32 tile of one slice:
// the gradient of the smooth part at the momentum point z is
// rho D_L (z - x) + s + grad R(z), with s = rho G + (1 - rho) g; the step
// uses the diagonal majorizer rho D_L + D_R and the nonnegativity
// projection.  Not last: v (holding v_{i-1}) <- v_i, zout <- v_i + mom
// (v_i - v_{i-1}).  Last: x <- v_i and the padded projector layouts.
struct InnerArgs {
    GeoK k;
    const float *z, *G, *g, *denom;
    float *v, *zout, *x, *XT, *XN;
    const DevScalars *sc;
    float beta, inv_delta2, mom;
    int nonneg;
    BatchStr bs;            // image b = blockIdx.z / nz
};

template <bool IS3D, bool LAST>
__global__ void __launch_bounds__(1024) inner_kernel(InnerArgs A)
{
    const GeoK &K = A.k;
    __shared__ float tile[32][33];
    const int k = (int)(blockIdx.z % (unsigned)K.nz);
    {
        // image bi of the batch
        const long long bi = blockIdx.z / (unsigned)K.nz;
        A.z += bi * A.bs.img;
        A.G += bi * A.bs.img;
        A.g += bi * A.bs.img;
        A.denom += bi * A.bs.img;
        A.v += bi * A.bs.img;
        if (A.zout) A.zout += bi * A.bs.img;
        A.x += bi * A.bs.img;
        A.XT += bi * A.bs.layT;
        A.XN += bi * A.bs.layN;
        A.sc += bi;
    }
    const DevScalars s = *A.sc;
    if (s.status) return;
    const float rho = (float)s.rho;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int i = blockIdx.x * 32 + tx, j = blockIdx.y * 32 + ty;
    const bool inside = i < K.nx && j < K.ny;
    float v = 0.0f;
    if (inside) {
        const long long idx = ((long long)k * K.ny + j) * K.nx + i;
        const float zv = A.z[idx], xv = A.x[idx], dl = (float)s.alpha * A.denom[idx];
        const float sv = fmaf(rho, A.G[idx], (1.0f - rho) * A.g[idx]);
        const float num = fmaf(rho * dl, zv - xv, sv) + reg_grad_at<IS3D>(K, A.z, i, j, k, A.beta, A.inv_delta2);
        const float den = fmaf(rho, dl, A.beta * reg_curv_sum(K, i, j, k));
        v = zv;
        if (den > 0.0f) {
            v = zv - num / den;
            if (A.nonneg) v = fmaxf(v, 0.0f);
        }
        if (LAST) {
            A.x[idx] = v;
            const long long n_idx = IS3D ? ((long long)j * K.slabN + (long long)(k + 2) * K.ldN + i + 2)
                                         : ((long long)j * K.ldN + i + 2);
            A.XN[n_idx] = v;
        } else {
            const float vp = A.v[idx];
            A.v[idx] = v;
            A.zout[idx] = fmaf(A.mom, v - vp, v);
        }
    }
    if (!LAST) return;
    tile[ty][tx] = v;
    __syncthreads();
    const int it = blockIdx.x * 32 + ty, jt = blockIdx.y * 32 + tx;
    if (it < K.nx && jt < K.ny) {
        const long long t_idx = IS3D ? ((long long)it * K.slabT + (long long)(k + 2) * K.ldT + jt + 2)
                                     : ((long long)it * K.ldT + jt + 2);
        A.XT[t_idx] = tile[tx][ty];
    }
}

template <bool IS3D>
hipError_t upd_dispatch(const lalm_plan *p, const UpdArgs &a, int mode, hipStream_t st)
{
    const int zs = (IS3D && !a.vout) ? UPD_ZS : 1;
    const long long ntile = (long long)((a.k.nx + 31) / 32) * ((a.k.ny + 31) / 32) * ((a.k.nz + zs - 1) / zs) * p->B;
    if (ntile > 0x7FFFFFF8LL) return hipErrorInvalidValue;
    dim3 blk(32, 32), grd((unsigned)((ntile + 7) / 8 * 8));   // padded to the eight XCDs
    constexpr int ZL = IS3D ? UPD_ZS : 1;                        // launches that store the layouts
    if (mode == UPD_LAYOUT) return klaunch(p, update_kernel<IS3D, UPD_LAYOUT, ZL>, grd, blk, st, a);
    if (mode == UPD_ONES) return klaunch(p, update_kernel<IS3D, UPD_ONES, ZL>, grd, blk, st, a);
    if (a.vout) return klaunch(p, update_kernel<IS3D, UPD_STEP, 1>, grd, blk, st, a);
    return klaunch(p, update_kernel<IS3D, UPD_STEP, ZL>, grd, blk, st, a);
}

__global__ void set_scalars_kernel(DevScalars *sc, long long l, double rho, long long step, double alpha)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->rho = rho;
        sc->xi = 0.0;
        sc->l = l;
        sc->step = step;
        sc->status = 0;
        sc->sel = 0;
        sc->alpha = alpha;
    }
}

// ---------------------------------------------------------------- Barzilai-Borwein
//
// <s, y> and <s, D_L s> with s = x - x_prev, y = grad - grad_prev, per block
// in FP64 (grid-stride, fixed order), then x_prev, grad_prev <- x, grad.
constexpr int BB_BLOCKS = 1024;

__global__ void __launch_bounds__(256) bb_dot_kernel(const float *x, const float *grad, float *xp, float *gp,
                                                     const float *denom, long long n, int compute, double *part,
                                                     long long part_stride)
{
    __shared__ double s_w[2][4];
    const int tid = threadIdx.x;
    {
        // image bi of the batch (n voxels each)
        const long long bi = blockIdx.y;
        x += bi * n;
        grad += bi * n;
        xp += bi * n;
        gp += bi * n;
        denom += bi * n;
        part += bi * part_stride;
    }
    double sy = 0.0, sls = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + tid; i < n; i += (long long)gridDim.x * 256) {
        const float xv = x[i], gv = grad[i];
        if (compute) {
            const double sv = (double)xv - (double)xp[i];
            sy += sv * ((double)gv - (double)gp[i]);
            sls += (double)denom[i] * sv * sv;
        }
        xp[i] = xv;
        gp[i] = gv;
    }
    if (!compute) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sy += __shfl_xor(sy, o, 64);
        sls += __shfl_xor(sls, o, 64);
    }
    if ((tid & 63) == 0) {
        s_w[0][tid >> 6] = sy;
        s_w[1][tid >> 6] = sls;
    }
    __syncthreads();
    if (tid == 0) {
        part[blockIdx.x] = (s_w[0][0] + s_w[0][1]) + (s_w[0][2] + s_w[0][3]);
        part[BB_BLOCKS + blockIdx.x] = (s_w[1][0] + s_w[1][1]) + (s_w[1][2] + s_w[1][3]);
    }
}

// alpha = min(1, <s,y> / <s,D_L s>), at least alpha_min; 1 without curvature
// information (non-positive sums).  Written into the current scalar record.
__global__ void __launch_bounds__(256) bb_finalize_kernel(const double *part, DevScalars *sc, double alpha_min,
                                                          long long part_stride)
{
    __shared__ double s_w[4];
    part += (long long)blockIdx.x * part_stride;     // one block per image
    sc += blockIdx.x;
    if (sc->status) return;
    const int tid = threadIdx.x;
    const double sy = fixed_sum_256(part, BB_BLOCKS, tid, s_w);
    const double sls = fixed_sum_256(part + BB_BLOCKS, BB_BLOCKS, tid, s_w);
    if (tid == 0) sc->alpha = (sy > 0.0 && sls > 0.0) ? fmin(1.0, fmax(alpha_min, sy / sls)) : 1.0;
}

}  // namespace

hipError_t launch_fp(const lalm_plan *p, int64_t slot0, int nview, const float *y, const float *w,
                     float *out, int mode, int64_t part_off, int64_t *n_blocks_out,
                     int check_status, hipStream_t st, int ray_scaled, int64_t yw_stride, int64_t out_stride)
{
    FPArgs a;
    a.k = p->k;
    a.rays = p->d_rays + slot0 * p->nb;
    a.raysz = p->is3d ? p->d_raysz + slot0 * p->nb : nullptr;
    a.views = p->d_views + slot0;
    a.rowv = p->d_rowv;
    a.rowf = p->d_rowf;
    a.XT = p->d_xt;
    a.XN = p->d_xn;
    a.nrays = (long long)nview * p->rays_per_view;
    a.y = y;
    a.w = w;
    a.out = out;
    a.partials = p->d_partials + part_off;
    a.st_sc = check_status ? cur_sc(p) : nullptr;
    a.XT1 = a.XN1 = nullptr;
    a.sc_in = nullptr;
    a.sc_out = nullptr;
    a.dec_part = nullptr;
    a.dec_n = 0;
    a.cont = ContArgs{};
    a.ray_scaled = ray_scaled;
    a.bs = batch_str(p);
    a.s_yw = yw_stride;
    a.s_out = out_stride;
    long long nblk = (a.nrays + 63) / 64;
    if (n_blocks_out) *n_blocks_out = nblk;
    if (nblk == 0) return hipSuccess;
    return p->is3d ? fp_dispatch<true>(p, a, p->fp_nseg, mode, nblk, st)
                   : fp_dispatch<false>(p, a, p->fp_nseg, mode, nblk, st);
}

hipError_t launch_fp_decide(const lalm_plan *p, int64_t slot0, int nview, const float *y, const float *w,
                            float *out, const ContArgs &cont, hipStream_t st, int64_t yw_stride,
                            int64_t out_stride)
{
    if (p->is3d || !p->d_xt1 || !p->d_xn1) return hipErrorInvalidValue;
    FPArgs a;
    a.k = p->k;
    a.rays = p->d_rays + slot0 * p->nb;
    a.raysz = nullptr;
    a.views = p->d_views + slot0;
    a.rowv = p->d_rowv;
    a.rowf = p->d_rowf;
    a.XT = p->d_xt;
    a.XN = p->d_xn;
    a.XT1 = p->d_xt1;
    a.XN1 = p->d_xn1;
    a.nrays = (long long)nview * p->rays_per_view;
    a.y = y;
    a.w = w;
    a.out = out;
    a.partials = nullptr;
    a.st_sc = nullptr;
    a.sc_in = cur_sc(p);
    a.sc_out = nxt_sc(p);
    a.dec_part = p->d_partials;
    a.dec_n = p->bp_nblocks;
    a.cont = cont;
    a.ray_scaled = 0;       // 2D residuals carry no ray scale
    a.bs = batch_str(p);
    a.s_yw = yw_stride;
    a.s_out = out_stride;
    const long long nblk = (a.nrays + 63) / 64;
    if (nblk == 0) return hipErrorInvalidValue;     // every subset holds a view
    const hipError_t e = fp_dispatch<false>(p, a, p->fp_nseg, 2, nblk, st);
    p->sc_cur ^= 1;
    return e;
}

hipError_t launch_update(const lalm_plan *p, int mode, float *x, const float *G, const float *g,
                         const float *denom, float beta, int nonneg, const ContArgs *cont, hipStream_t st,
                         float *vout, float *zout)
{
    UpdArgs a;
    a.k = p->k;
    a.x = x;
    a.G = G;
    a.g = g;
    a.gradR = p->d_gradR;
    a.denom = denom;
    a.XT = p->d_xt;
    a.XN = p->d_xn;
    a.sc = cur_sc(p);
    a.beta = beta;
    a.nonneg = nonneg;
    a.do_finalize = (mode == UPD_STEP && cont) ? 1 : 0;
    a.partials = p->d_partials;
    a.nblocks = p->bp_nblocks;
    a.sc_out = nxt_sc(p);
    if (a.do_finalize) a.cont = *cont;
    else a.cont = ContArgs{};
    a.vout = mode == UPD_STEP ? vout : nullptr;
    a.zout = mode == UPD_STEP ? zout : nullptr;
    a.bs = batch_str(p);
    a.nimg = p->B;
    hipError_t e = p->is3d ? upd_dispatch<true>(p, a, mode, st) : upd_dispatch<false>(p, a, mode, st);
    if (a.do_finalize) p->sc_cur ^= 1;
    return e;
}

hipError_t launch_inner(const lalm_plan *p, const float *z, float *v, float *zout, float *x, const float *G,
                        const float *g, const float *denom, float beta, float inv_delta2, float mom, int nonneg,
                        bool last, hipStream_t st)
{
    InnerArgs a;
    a.k = p->k;
    a.z = z;
    a.G = G;
    a.g = g;
    a.denom = denom;
    a.v = v;
    a.zout = zout;
    a.x = x;
    a.XT = p->d_xt;
    a.XN = p->d_xn;
    a.sc = cur_sc(p);
    a.beta = beta;
    a.inv_delta2 = inv_delta2;
    a.mom = mom;
    a.nonneg = nonneg;
    a.bs = batch_str(p);
    dim3 blk(32, 32), grd((p->nx + 31) / 32, (p->ny + 31) / 32, (unsigned)(p->nz * p->B));
    if (p->is3d) return last ? klaunch(p, inner_kernel<true, true>, grd, blk, st, a)
                             : klaunch(p, inner_kernel<true, false>, grd, blk, st, a);
    return last ? klaunch(p, inner_kernel<false, true>, grd, blk, st, a)
                : klaunch(p, inner_kernel<false, false>, grd, blk, st, a);
}

hipError_t launch_set_scalars(const lalm_plan *p, int b, long long l, double rho, long long step, double alpha,
                              hipStream_t st)
{
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, st, cur_sc(p) + b, l, rho, step, alpha);
    return hipGetLastError();
}

hipError_t launch_bb(const lalm_plan *p, const float *x, const float *grad, float *x_prev, float *grad_prev,
                     const float *denom, bool compute, double alpha_min, hipStream_t st)
{
    // the last 2 x BB_BLOCKS partial slots, above any back-projection's block partials
    double *part = p->d_partials + p->n_partials - 2 * BB_BLOCKS;
    const long long n = (long long)p->nx * p->ny * p->nz;
    hipLaunchKernelGGL(bb_dot_kernel, dim3(BB_BLOCKS, p->B), dim3(256), 0, st, x, grad, x_prev, grad_prev, denom, n,
                       compute ? 1 : 0, part, (long long)p->n_partials);
    if (compute) hipLaunchKernelGGL(bb_finalize_kernel, dim3(p->B), dim3(256), 0, st, (const double *)part, cur_sc(p),
                                    alpha_min, (long long)p->n_partials);
    return hipGetLastError();
}

}  // namespace lalm
