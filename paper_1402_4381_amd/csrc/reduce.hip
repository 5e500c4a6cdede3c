// FP64 reductions for the monitors: cost (data term partials come from the
// forward projector, regularizer value here), inner products for the adjoint
// test and the ROI RMS difference.  Every reduction uses a fixed grid and a
// fixed summation order, so results are bit-reproducible.
#include <mutex>

#include "lalm_internal.h"

namespace lalm {
namespace {

constexpr int kRedBlocks = 1024;

__device__ inline double tree_256(double v, double *s)
{
    const int tid = threadIdx.x;
    s[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) s[tid] += s[tid + w];
        __syncthreads();
    }
    return s[0];
}

__global__ void __launch_bounds__(256) sum_partials_kernel(const double *p, long long n, double *out,
                                                           double scale)
{
    __shared__ double s[256];
    double v = 0.0;
    for (long long t = threadIdx.x; t < n; t += 256) v += p[t];
    const double tot = tree_256(v, s);
    if (threadIdx.x == 0) out[0] = scale * tot;
}

__global__ void __launch_bounds__(256) dot_kernel(const float *a, const float *b, long long n,
                                                  double *part)
{
    __shared__ double s[256];
    double v = 0.0;
    const long long stride = (long long)gridDim.x * 256;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += stride)
        v += (double)a[t] * (double)b[t];
    const double tot = tree_256(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// psi(t) = delta^2 (sqrt(1 + (t/delta)^2) - 1) = t^2 / (sqrt(1 + (t/delta)^2) + 1)
__device__ inline double psi64(double t, double delta)
{
    const double u = t / delta;
    return t * t / (sqrt(1.0 + u * u) + 1.0);
}

// R(x): every neighbour pair once (offsets in the lexicographic upper half).
__global__ void __launch_bounds__(256) reg_value_kernel(GeoK K, const float *x, double beta,
                                                        double delta, double *part)
{
    __shared__ double s[256];
    const long long n = (long long)K.nx * K.ny * K.nz;
    const long long plane = (long long)K.nx * K.ny;
    const long long stride = (long long)gridDim.x * 256;
    double v = 0.0;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += stride) {
        const int i = (int)(t % K.nx), j = (int)((t / K.nx) % K.ny), k = (int)(t / plane);
        const double xc = x[t];
        const int zlo = K.is3d ? -1 : 0, zhi = K.is3d ? 1 : 0;
        for (int dz = zlo; dz <= zhi; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    // upper half: (dz, dy, dx) > (0, 0, 0) lexicographically
                    if (dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx <= 0)))) continue;
                    const int ii = i + dx, jj = j + dy, kk = k + dz;
                    if (ii < 0 || ii >= K.nx || jj < 0 || jj >= K.ny || kk < 0 || kk >= K.nz) continue;
                    const int nz_ = (dx != 0) + (dy != 0) + (dz != 0);
                    const double kap = 1.0 / sqrt((double)nz_);
                    const double xn = x[t + (long long)dz * plane + (long long)dy * K.nx + dx];
                    v += kap * psi64(xc - xn, delta);
                }
    }
    const double tot = tree_256(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = beta * tot;
}

__global__ void __launch_bounds__(256) rmsd_kernel(GeoK K, const float *a, const float *b,
                                                   double radius, double *part, double *cnt)
{
    __shared__ double s[256];
    const long long n = (long long)K.nx * K.ny * K.nz;
    const long long stride = (long long)gridDim.x * 256;
    double v = 0.0, c = 0.0;
    const double r2 = radius * radius;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n; t += stride) {
        const int i = (int)(t % K.nx), j = (int)((t / K.nx) % K.ny);
        const double X = (i - (K.nx - 1) / 2.0) * (double)K.dx;
        const double Y = (j - (K.ny - 1) / 2.0) * (double)K.dy;
        if (X * X + Y * Y <= r2) {
            const double d = (double)a[t] - (double)b[t];
            v += d * d;
            c += 1.0;
        }
    }
    const double tv = tree_256(v, s);
    __syncthreads();
    const double tc = tree_256(c, s);
    if (threadIdx.x == 0) { part[blockIdx.x] = tv; cnt[blockIdx.x] = tc; }
}

__global__ void rmsd_final_kernel(const double *part, const double *cnt, int n, double *out)
{
    if (threadIdx.x != 0) return;
    double v = 0.0, c = 0.0;
    for (int t = 0; t < n; ++t) { v += part[t]; c += cnt[t]; }
    out[0] = c > 0 ? sqrt(v / c) : 0.0;
}

__global__ void combine_cost_kernel(double *out3, const double *data, const double *reg)
{
    if (threadIdx.x != 0) return;
    const double d = data[0], r = reg[0];
    out3[0] = d + r;
    out3[1] = d;
    out3[2] = r;
}

}  // namespace

hipError_t launch_sum_partials(const double *part, int64_t n, double *out, double scale,
                               hipStream_t st)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, part, (long long)n, out, scale);
    return hipGetLastError();
}

hipError_t launch_dot(const lalm_plan *p, const float *a, const float *b, int64_t n, double *out,
                      hipStream_t st)
{
    hipLaunchKernelGGL(dot_kernel, dim3(kRedBlocks), dim3(256), 0, st, a, b, (long long)n, p->d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(p->d_partials, kRedBlocks, out, 1.0, st);
}

hipError_t launch_reg_value(const lalm_plan *p, const float *x, double beta, double delta,
                            double *out, hipStream_t st)
{
    hipLaunchKernelGGL(reg_value_kernel, dim3(kRedBlocks), dim3(256), 0, st, p->k, x, beta, delta,
                       p->d_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(p->d_partials, kRedBlocks, out, 1.0, st);
}

hipError_t launch_rmsd(const lalm_plan *p, const float *a, const float *b, double radius,
                       double *out, hipStream_t st)
{
    hipLaunchKernelGGL(rmsd_kernel, dim3(kRedBlocks), dim3(256), 0, st, p->k, a, b, radius,
                       p->d_partials, p->d_partials + kRedBlocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rmsd_final_kernel, dim3(1), dim3(64), 0, st, p->d_partials,
                       p->d_partials + kRedBlocks, kRedBlocks, out);
    return hipGetLastError();
}

hipError_t launch_combine_cost(double *out3, const double *data, const double *reg, hipStream_t st)
{
    hipLaunchKernelGGL(combine_cost_kernel, dim3(1), dim3(64), 0, st, out3, data, reg);
    return hipGetLastError();
}

}  // namespace lalm

// ------------------------------------------------------------ no allocation
//
// lalm_dot_f64_noalloc: the dot product of lalm_dot_f64 for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops).  Its only scratch, the FP64 block partials, lives in a file-scope
// device array: one per GPU, held until the process ends, shared by every
// call on that GPU.  The host reaches it through the address
// hipGetSymbolAddress returns for the current device, never through the
// array's name.

static __device__ __align__(256) double scratch[lalm::kRedBlocks];

namespace {

constexpr int kMaxDevices = 64;
constexpr int64_t kNoallocMaxN = int64_t(1) << 40;    // elements per operand
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// This device's copy of the scratch array (looked up once per device).
hipError_t scratch_of_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" lalm_status lalm_dot_f64_noalloc(const float *a, const float *b, int64_t n, double *out_dev,
                                            hipStream_t st)
{
    if (!a || !b || !out_dev || n < 0) {
        lalm::set_error("lalm_dot_f64_noalloc: bad argument");
        return LALM_E_INVALID;
    }
    if (n > kNoallocMaxN) {
        lalm::set_error("lalm_dot_f64_noalloc: more than 2^40 elements");
        return LALM_E_INVALID;
    }
    double *part = nullptr;
    hipError_t e = scratch_of_current_device(&part);
    if (e != hipSuccess) {
        lalm::set_error(std::string("lalm_dot_f64_noalloc: scratch address: ") + hipGetErrorString(e));
        return LALM_E_HIP;
    }
    // the same kernels and grid as lalm_dot_f64: every block overwrites its
    // partial, so nothing needs clearing between calls
    hipLaunchKernelGGL(lalm::dot_kernel, dim3(lalm::kRedBlocks), dim3(256), 0, st, a, b, (long long)n, part);
    e = hipGetLastError();
    if (e == hipSuccess) e = lalm::launch_sum_partials(part, lalm::kRedBlocks, out_dev, 1.0, st);
    if (e != hipSuccess) {
        lalm::set_error(std::string("lalm_dot_f64_noalloc: ") + hipGetErrorString(e));
        return LALM_E_HIP;
    }
    return LALM_OK;
}
