// Initial image by filtered back-projection over one full turn: the image
// the paper's experiments start from (figure captions).  Textbook
// reconstructions for the arc (equiangular, cylindrical) detector:
//   2D fan beam   the data are weighted by D cos(gamma), filtered along the
//                 channels with the fan-beam Ram-Lak kernel
//                 g(n dg) = 1/2 (n dg / sin(n dg))^2 h(n dg), which is
//                 1/(8 dg^2) at n = 0, -1/(2 pi^2 sin^2(n dg)) at odd n and 0
//                 at even n, and back-projected with the weight 1/L^2 (L: the
//                 distance from the source) and linear interpolation in
//                 channel;
//   axial cone    FDK (Feldkamp, Davis & Kress): the weight also carries the
//                 cone angle of the row, dsd / sqrt(dsd^2 + v_r^2), every
//                 detector row is filtered on its own with the same kernel,
//                 and a voxel at height z takes the filtered value at the row
//                 height v = z dsd / L (L: the in-plane distance from the
//                 source), bilinear in (channel, row), with the weight 1/L^2.
#include "lalm_internal.h"

namespace lalm {
namespace {

constexpr int FBP_NBMAX = 4096;   // channels per view held in LDS

// Q[slot][row][b] = dg sum_k q[k] g(b - k), q[k] = y[slot][row][k] D cos(gamma_k) c_row
// with the cone weight c_row = dsd / sqrt(dsd^2 + v_row^2) (1 in 2D); one
// block per detector row of a view, the weighted row and the kernel table
// in LDS, each output summed over k in increasing order.
__global__ void __launch_bounds__(256) fbp_filter_kernel(const float *y, float *Q, int nb, double dg, double D,
                                                         double center, int nr, double dt, double dsd,
                                                         long long sino_elems)
{
    __shared__ float q[FBP_NBMAX];
    __shared__ float gk[FBP_NBMAX];
    const long long base = (long long)blockIdx.y * sino_elems + (long long)blockIdx.x * nb;   // image, row
    const double pi = 3.14159265358979323846;
    const double vr = ((double)(blockIdx.x % nr) - (nr - 1) / 2.0) * dt;
    const double Dc = vr == 0.0 ? D : D * (dsd / sqrt(dsd * dsd + vr * vr));
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        q[k] = (float)((double)y[base + k] * Dc * cos(((double)k - center) * dg));
        double g = 0.0;
        if (k == 0) {
            g = 1.0 / (8.0 * dg * dg);
        } else if (k & 1) {
            const double sn = sin((double)k * dg);
            g = -1.0 / (2.0 * pi * pi * sn * sn);
        }
        gk[k] = (float)g;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        float acc = 0.0f;
        for (int k = 0; k < nb; ++k) {
            const int d = b > k ? b - k : k - b;
            acc = fmaf(q[k], gk[d], acc);
        }
        Q[base + b] = (float)dg * acc;
    }
}

// x[j][i] = dbeta sum_views Q(gamma'(P)) / L(P)^2
__global__ void __launch_bounds__(256) fbp_backproject_kernel(GeoK K, const ViewRec *views, int nview,
                                                              const float *Q, float dbeta, float *x)
{
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y;
    Q += (long long)blockIdx.z * nview * K.nb;          // image of the batch
    x += (long long)blockIdx.z * K.nx * K.ny;
    if (i >= K.nx || j >= K.ny) return;
    const float X = fmaf((float)i, K.dx, K.x0), Y = fmaf((float)j, K.dy, K.y0);
    float acc = 0.0f;
    for (int v = 0; v < nview; ++v) {
        const ViewRec V = views[v];
        const float ddx = X - V.sx, ddy = Y - V.sy;
        const float dc = -(ddx * V.cb + ddy * V.sb);
        const float dp = ddx * V.sb - ddy * V.cb;
        const float bc = fmaf(atan2f(dp, dc), K.dsd_over_ds, K.bin_center);
        const float fl = floorf(bc);
        const int b0 = (int)fl;
        const float t = bc - fl;
        const float *row = Q + (long long)v * K.nb;
        float val = 0.0f;
        if (b0 >= 0 && b0 < K.nb) val = (1.0f - t) * row[b0];
        if (b0 + 1 >= 0 && b0 + 1 < K.nb) val = fmaf(t, row[b0 + 1], val);
        acc += val / fmaf(ddx, ddx, ddy * ddy);
    }
    x[(long long)j * K.nx + i] = dbeta * acc;
}

constexpr int FDK_KZ = 8;   // slices per thread of the FDK back-projection

// x[k][j][i] = dbeta sum_views Q(gamma'(P), v'(P)) / L(P)^2 for the axial
// cone beam (source at z = 0): a thread owns FDK_KZ slices of one column and
// shares the in-plane part (fan angle, 1/L) of each view among them.
__global__ void __launch_bounds__(256) fdk_backproject_kernel(GeoK K, const ViewRec *views, int nview,
                                                              const float *Q, float dbeta, float rows_per_mm,
                                                              float *x)
{
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y;
    const unsigned nzb = (unsigned)(K.nz + FDK_KZ - 1) / FDK_KZ;
    const int kb = (int)(blockIdx.z % nzb) * FDK_KZ;
    {
        const long long bi = blockIdx.z / nzb;           // image of the batch
        Q += bi * nview * K.nr * (long long)K.nb;
        x += bi * K.nx * K.ny * (long long)K.nz;
    }
    if (i >= K.nx || j >= K.ny) return;
    const float X = fmaf((float)i, K.dx, K.x0), Y = fmaf((float)j, K.dy, K.y0);
    float Z[FDK_KZ], acc[FDK_KZ];
#pragma unroll
    for (int t = 0; t < FDK_KZ; ++t) {
        Z[t] = ((float)(kb + t) - 0.5f * (float)(K.nz - 1)) * K.dz;
        acc[t] = 0.0f;
    }
    const long long per_view = (long long)K.nr * K.nb;
    for (int v = 0; v < nview; ++v) {
        const ViewRec V = views[v];
        const float ddx = X - V.sx, ddy = Y - V.sy;
        const float dc = -(ddx * V.cb + ddy * V.sb);
        const float dp = ddx * V.sb - ddy * V.cb;
        const float bc = fmaf(atan2f(dp, dc), K.dsd_over_ds, K.bin_center);
        const float fl = floorf(bc);
        const int b0 = (int)fl;
        const float tb = bc - fl;
        const bool in0 = b0 >= 0 && b0 < K.nb, in1 = b0 + 1 >= 0 && b0 + 1 < K.nb;
        const float L2 = fmaf(ddx, ddx, ddy * ddy);
        const float w = dbeta / L2;
        const float rscale = rows_per_mm / sqrtf(L2);     // detector rows per mm of z at this column
        const float *Qv = Q + (long long)v * per_view;
#pragma unroll
        for (int t = 0; t < FDK_KZ; ++t) {
            const float rc = fmaf(Z[t], rscale, K.row_center);
            const float flr = floorf(rc);
            const int r0 = (int)flr;
            const float tr = rc - flr;
            float val = 0.0f;
            if (r0 >= 0 && r0 < K.nr) {
                const float *row = Qv + (long long)r0 * K.nb;
                float s = 0.0f;
                if (in0) s = (1.0f - tb) * row[b0];
                if (in1) s = fmaf(tb, row[b0 + 1], s);
                val = (1.0f - tr) * s;
            }
            if (r0 + 1 >= 0 && r0 + 1 < K.nr) {
                const float *row = Qv + (long long)(r0 + 1) * K.nb;
                float s = 0.0f;
                if (in0) s = (1.0f - tb) * row[b0];
                if (in1) s = fmaf(tb, row[b0 + 1], s);
                val = fmaf(tr, s, val);
            }
            acc[t] = fmaf(w, val, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < FDK_KZ; ++t) {
        const int k = kb + t;
        if (k < K.nz) x[((long long)k * K.ny + j) * K.nx + i] = acc[t];
    }
}

}  // namespace

hipError_t launch_fbp(const lalm_plan *p, const float *y, float *x, hipStream_t st)
{
    const lalm_geometry &g = p->g;
    const double dg = g.ds / g.dsd;
    const double center = (p->nb - 1) / 2.0 + g.channel_offset;
    const int nr = p->is3d ? p->nr : 1;
    hipLaunchKernelGGL(fbp_filter_kernel, dim3((unsigned)(p->nv * nr), p->B), dim3(256), 0, st, y, p->d_fbpq, p->nb,
                       dg, g.dso, center, nr, g.dt, g.dsd, (long long)p->nv * nr * p->nb);
    const double dbeta = 2.0 * 3.14159265358979323846 / g.n_views_per_turn;
    if (!p->is3d) {
        dim3 blk(32, 8), grd((p->nx + 31) / 32, (p->ny + 7) / 8, p->B);
        hipLaunchKernelGGL(fbp_backproject_kernel, grd, blk, 0, st, p->k, (const ViewRec *)p->d_views, p->nv,
                           (const float *)p->d_fbpq, (float)dbeta, x);
    } else {
        dim3 blk(32, 8), grd((p->nx + 31) / 32, (p->ny + 7) / 8, (unsigned)((p->nz + FDK_KZ - 1) / FDK_KZ * p->B));
        hipLaunchKernelGGL(fdk_backproject_kernel, grd, blk, 0, st, p->k, (const ViewRec *)p->d_views, p->nv,
                           (const float *)p->d_fbpq, (float)dbeta, (float)(g.dsd / g.dt), x);
    }
    return hipGetLastError();
}

int fbp_max_bins() { return FBP_NBMAX; }

}  // namespace lalm
