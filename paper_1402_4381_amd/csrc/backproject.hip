// Matched back-projection (deterministic voxel-driven gather) and the fused
// OS-LALM epilogue.
//
// Each thread owns one voxel column (i, j) and, in 3D, KZ consecutive slices.
// For every view of the subset it finds the detector channels whose rays can
// reach the voxel (the angular window of a disc of radius max(dx, dy) around
// the voxel centre, seen from the source) and evaluates, for each candidate,
// the forward projector's own interpolation weight from the same FP32 table
// entries with the same fused multiply-adds.  The result is the exact
// transpose of the forward projector up to the order of FP32 additions, with
// no atomics: every voxel is written by one thread, in a fixed order.
//
// Epilogues (one pass over the image, no extra launch):
//   BP_PLAIN  out = scale * A_m' r   (or +=)
//   BP_INIT   G = g = M A_m' r, grad R(x); FP64 sum of G^2 (finite check)
//   BP_STEP   G+ = M A_m' r;  xi partial (g - G+)(G+ - G) in FP64;
//             g <- (rho G+ + g) / (rho + 1);  G <- G+;  grad R(x)
// The last block to finish (device-wide counter) reduces the FP64 partials in
// a fixed order and performs the continuation update of Sec. III-B.
#include "lalm_internal.h"

namespace lalm {
namespace {

constexpr int KZ3 = 8;   // slices per thread in 3D

struct BPArgs {
    GeoK k;
    const RayRec *rays;
    const RayRecZ *raysz;
    const ViewRec *views;
    const float *rowv, *rowf;
    int nview;
    const float *r;
    BpEpi e;
    double *partials;
    unsigned int *counter;
    DevScalars *sc;
    int nblocks;
};

// d psi / dt for the hyperbola potential: t / sqrt(1 + (t/delta)^2)
__device__ inline float dpsi(float t, float inv_delta2)
{
    return t * rsqrtf(fmaf(t * t, inv_delta2, 1.0f));
}

// grad R at voxel (i, j, k): beta sum_{n in N} kappa psi'(x_c - x_n)
template <bool IS3D>
__device__ float reg_grad_at(const GeoK &K, const float *x, int i, int j, int k, float beta,
                             float inv_delta2)
{
    const long long plane = (long long)K.nx * K.ny;
    const long long c = (long long)k * plane + (long long)j * K.nx + i;
    const float xc = x[c];
    const float r2 = 0.70710678118654752f, r3 = 0.57735026918962576f;
    float s = 0.0f;
    const int zlo = IS3D ? -1 : 0, zhi = IS3D ? 1 : 0;
#pragma unroll
    for (int dz = zlo; dz <= zhi; ++dz) {
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii < 0 || ii >= K.nx || jj < 0 || jj >= K.ny || kk < 0 || kk >= K.nz) continue;
                const int n = (dx != 0) + (dy != 0) + (dz != 0);
                const float kap = n == 1 ? 1.0f : (n == 2 ? r2 : r3);
                const float xn = x[c + (long long)dz * plane + (long long)dy * K.nx + dx];
                s = fmaf(kap, dpsi(xc - xn, inv_delta2), s);
            }
        }
    }
    return beta * s;
}

__device__ inline double block_sum_256(double v, double *lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if ((tid & 63) == 0) lds[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (tid == 0) t = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    return t;   // valid in thread 0
}

template <bool IS3D, int MODE>
__global__ void __launch_bounds__(256) bp_kernel(BPArgs A)
{
    constexpr int KZ = IS3D ? KZ3 : 1;
    const GeoK &K = A.k;
    if (MODE != BP_PLAIN && A.sc->status) return;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + ty * 32;
    const int i = blockIdx.x * 32 + tx, j = blockIdx.y * 8 + ty;
    const int kb = blockIdx.z * KZ;
    const bool inside = i < K.nx && j < K.ny;

    __shared__ float s_rowv[256], s_rowf[256];
    __shared__ double s_red[4];
    __shared__ double s_tree[256];
    __shared__ int s_last;
    if (IS3D) {
        for (int t = tid; t < K.nr; t += 256) { s_rowv[t] = A.rowv[t]; s_rowf[t] = A.rowf[t]; }
        __syncthreads();
    }

    float acc[KZ];
#pragma unroll
    for (int t = 0; t < KZ; ++t) acc[t] = 0.0f;

    if (inside) {
        const float X = fmaf((float)i, K.dx, K.x0), Y = fmaf((float)j, K.dy, K.y0);
        for (int kv = 0; kv < A.nview; ++kv) {
            const ViewRec V = A.views[kv];
            const float ddx = X - V.sx, ddy = Y - V.sy;
            const float dc = -(ddx * V.cb + ddy * V.sb);
            const float dp = ddx * V.sb - ddy * V.cb;
            const float gam = atan2f(dp, dc);
            const float bc = fmaf(gam, K.dsd_over_ds, K.bin_center);
            const float dist = sqrtf(fmaf(ddx, ddx, ddy * ddy));
            const float hw = dist > 2.0f * K.dmax ? K.dmax / (dist - K.dmax) * K.dsd_over_ds + 0.05f
                                                  : (float)K.nb;
            const int b0 = max(0, (int)ceilf(bc - hw));
            const int b1 = min(K.nb - 1, (int)floorf(bc + hw));
            const RayRec *R = A.rays + (long long)kv * K.nb;
            for (int b = b0; b <= b1; ++b) {
                const RayRec rr = R[b];
                const bool ydom = meta_ydom(rr.meta);
                const int s = ydom ? j : i, o = ydom ? i : j;
                const float eta = fmaf((float)s, rr.c, rr.a);
                const float fl = floorf(eta);
                const float f = eta - fl;
                const int j0 = (int)fl;
                const float wxy = (j0 == o) ? (1.0f - f) : ((j0 + 1 == o) ? f : 0.0f);
                if (wxy == 0.0f) continue;
                if (!IS3D) {
                    acc[0] = fmaf(wxy * rr.sc, A.r[(long long)kv * K.nb + b], acc[0]);
                } else {
                    const RayRecZ rz = A.raysz[(long long)kv * K.nb + b];
                    const float qz = fmaf((float)s, rz.k, rz.m);
                    const float inv = K.inv_dt / qz;     // detector rows per slice
                    const float base = wxy * rr.sc;
                    const float *rcol = A.r + (long long)kv * K.nr * K.nb + b;
#pragma unroll
                    for (int t = 0; t < KZ; ++t) {
                        const int k = kb + t;
                        if (k >= K.nz) break;
                        const int r0 = max(0, (int)ceilf(fmaf((float)(k - 1) - V.z0, inv, K.row_center) - 0.01f));
                        const int r1 = min(K.nr - 1, (int)floorf(fmaf((float)(k + 1) - V.z0, inv, K.row_center) + 0.01f));
                        for (int rw = r0; rw <= r1; ++rw) {
                            const float zeta = fmaf(s_rowv[rw], qz, V.z0);
                            const float zl = floorf(zeta);
                            const float h = zeta - zl;
                            const int k0 = (int)zl;
                            const float wz = (k0 == k) ? (1.0f - h) : ((k0 + 1 == k) ? h : 0.0f);
                            if (wz != 0.0f)
                                acc[t] = fmaf(base * wz * s_rowf[rw], rcol[(long long)rw * K.nb], acc[t]);
                        }
                    }
                }
            }
        }
    }

    // ---------------------------------------------------------------- epilogue
    double part = 0.0;
    const float inv_delta2 = A.e.inv_delta2;
    const float rho = (MODE == BP_STEP) ? (float)A.sc->rho : 1.0f;
    if (inside) {
#pragma unroll
        for (int t = 0; t < KZ; ++t) {
            const int k = kb + t;
            if (k >= K.nz) break;
            const long long idx = ((long long)k * K.ny + j) * K.nx + i;
            if (MODE == BP_PLAIN) {
                const float v = A.e.scale * acc[t];
                A.e.out[idx] = A.e.accumulate ? A.e.out[idx] + v : v;
            } else if (MODE == BP_INIT) {
                const float Gv = A.e.scale * acc[t];
                A.e.G[idx] = Gv;
                A.e.g[idx] = Gv;
                A.e.out[idx] = reg_grad_at<IS3D>(K, A.e.x, i, j, k, A.e.beta, inv_delta2);
                part += (double)Gv * (double)Gv;
            } else {
                const float Gn = A.e.scale * acc[t];
                const float Go = A.e.G[idx], gv = A.e.g[idx];
                part += ((double)gv - (double)Gn) * ((double)Gn - (double)Go);
                A.e.g[idx] = fmaf(rho, Gn, gv) / (rho + 1.0f);
                A.e.G[idx] = Gn;
                A.e.out[idx] = reg_grad_at<IS3D>(K, A.e.x, i, j, k, A.e.beta, inv_delta2);
            }
        }
    }
    if (MODE == BP_PLAIN) return;

    const double bsum = block_sum_256(part, s_red);
    const int blin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (tid == 0) {
        __hip_atomic_store(&A.partials[blin], bsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned prev = atomicAdd(A.counter, 1u);
        s_last = (prev == (unsigned)A.nblocks - 1u);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // fixed-order reduction of the block partials
    double v = 0.0;
    for (int t = tid; t < A.nblocks; t += 256)
        v += __hip_atomic_load(&A.partials[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_tree[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) s_tree[tid] += s_tree[tid + w];
        __syncthreads();
    }
    if (tid != 0) return;
    const double total = s_tree[0];
    DevScalars *sc = A.sc;
    const ContArgs &C = A.e.cont;
    if (MODE == BP_INIT) {
        if (!isfinite(total)) sc->status = 1;
    } else {
        const long long jstep = sc->step;
        const double rho_used = sc->rho;
        bool restart = false;
        if (!isfinite(total)) {
            sc->status = 1;
        } else if (C.continuation) {
            restart = total > 0.0;
            if (C.forced && jstep < C.forced_len) restart = C.forced[jstep] != 0;
            const long long l = restart ? 0 : sc->l + 1;
            sc->l = l;
            double nr;
            if (l == 0) {
                nr = 1.0;
            } else {
                const double pi = 3.14159265358979323846;
                const double a = pi / (2.0 * (double)(l + 1));
                nr = fmax(pi / (double)(l + 1) * sqrt(1.0 - a * a), C.rho_min);
            }
            sc->rho = nr;
        }
        sc->xi = total;
        if (jstep < C.st_cap) {
            if (C.st_rho) C.st_rho[jstep] = rho_used;
            if (C.st_xi) C.st_xi[jstep] = total;
            if (C.st_restart) C.st_restart[jstep] = restart ? 1 : 0;
        }
        sc->step = jstep + 1;
    }
    *A.counter = 0u;
}

template <bool IS3D>
hipError_t bp_dispatch(const BPArgs &a, int mode, dim3 grd, hipStream_t st)
{
    dim3 blk(32, 8);
    if (mode == BP_PLAIN) hipLaunchKernelGGL((bp_kernel<IS3D, BP_PLAIN>), grd, blk, 0, st, a);
    else if (mode == BP_INIT) hipLaunchKernelGGL((bp_kernel<IS3D, BP_INIT>), grd, blk, 0, st, a);
    else hipLaunchKernelGGL((bp_kernel<IS3D, BP_STEP>), grd, blk, 0, st, a);
    return hipGetLastError();
}

template <bool IS3D>
__global__ void __launch_bounds__(256) reg_grad_kernel(GeoK K, const float *x, float *out, float beta,
                                                       float inv_delta2)
{
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y, k = blockIdx.z;
    if (i >= K.nx || j >= K.ny) return;
    out[((long long)k * K.ny + j) * K.nx + i] = reg_grad_at<IS3D>(K, x, i, j, k, beta, inv_delta2);
}

}  // namespace

hipError_t launch_bp(const lalm_plan *p, int64_t slot0, int nview, const float *r, int mode,
                     const BpEpi &e, hipStream_t st)
{
    BPArgs a;
    a.k = p->k;
    a.rays = p->d_rays + slot0 * p->nb;
    a.raysz = p->is3d ? p->d_raysz + slot0 * p->nb : nullptr;
    a.views = p->d_views + slot0;
    a.rowv = p->d_rowv;
    a.rowf = p->d_rowf;
    a.nview = nview;
    a.r = r;
    a.e = e;
    if (mode != BP_PLAIN) a.e.out = p->d_gradR;
    a.partials = p->d_partials;
    a.counter = p->d_counter;
    a.sc = p->d_sc;
    const int kz = p->is3d ? KZ3 : 1;
    dim3 grd((p->nx + 31) / 32, (p->ny + 7) / 8, (p->nz + kz - 1) / kz);
    a.nblocks = (int)(grd.x * grd.y * grd.z);
    return p->is3d ? bp_dispatch<true>(a, mode, grd, st) : bp_dispatch<false>(a, mode, grd, st);
}

hipError_t launch_reg_grad(const lalm_plan *p, const float *x, float beta, float inv_delta2,
                           hipStream_t st)
{
    dim3 blk(32, 8), grd((p->nx + 31) / 32, (p->ny + 7) / 8, p->nz);
    if (p->is3d)
        hipLaunchKernelGGL((reg_grad_kernel<true>), grd, blk, 0, st, p->k, x, p->d_gradR, beta, inv_delta2);
    else
        hipLaunchKernelGGL((reg_grad_kernel<false>), grd, blk, 0, st, p->k, x, p->d_gradR, beta, inv_delta2);
    return hipGetLastError();
}

}  // namespace lalm
