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
// Every block writes its FP64 partial sum; a one-block finalize kernel then
// reduces the partials in a fixed order and performs the continuation update
// of Sec. III-B (the kernel boundary orders the partial stores before the
// reduction without a device-scope fence per block).
#include "lalm_internal.h"

namespace lalm {
namespace {

constexpr int KZ3 = 8;   // slices per thread in 3D
constexpr int BP3_RW = 2;   // detector rows per slice whose gathers go out together

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
    DevScalars *sc;
    int nblocks;
    float *part;       // 2D: back-projection of the x-dominant rays
    float *part2;      // 2D: back-projection of the y-dominant rays
    int check_status;  // 2D line kernel: skip when a non-finite indicator was met
    BatchStr bs;       // batch: image b's residual starts at r + b e.r_stride
};

// Pointers of BPArgs moved to image bi of the batch.
__device__ inline void bp_args_at(BPArgs &A, long long bi)
{
    A.r += bi * A.e.r_stride;
    if (A.e.out) A.e.out += bi * A.bs.img;
    if (A.e.G) A.e.G += bi * A.bs.img;
    if (A.e.g) A.e.g += bi * A.bs.img;
    if (A.e.x) A.e.x += bi * A.bs.img;
    if (A.partials) A.partials += bi * A.bs.part;
    if (A.sc) A.sc += bi;
    if (A.part) A.part += bi * A.bs.img;
    if (A.part2) A.part2 += bi * A.bs.img;
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

// atan(t) = t P(t^2) on [0, 1] with a degree-5 polynomial P fitted by
// reweighted least squares on Chebyshev nodes (max error 1.7e-6 rad), and
// atan(t) = pi/2 - atan(1/t) above 1.  Used only to bound channel windows;
// the window margin covers its error.  (The 3D kernel and the 2D line
// kernel both use it.)  The window set-up also takes the hardware
// reciprocal and square root (v_rcp_f32, v_sqrt_f32, about 1 ulp) where a
// correctly rounded division or root would cost a dozen instructions: their
// results only place windows that carry a margin of at least 0.01 channel or
// row, far above those errors.
__device__ inline float atan_window(float t)
{
    const float at = fabsf(t);
    const bool big = at > 1.0f;
    const float z = big ? __builtin_amdgcn_rcpf(at) : at;   // hardware reciprocal, 1 ulp
    const float z2 = z * z;
    float p = fmaf(z2, -0.011719409376382828f, 0.05264794081449509f);
    p = fmaf(z2, p, -0.11642685532569885f);
    p = fmaf(z2, p, 0.19354040920734406f);
    p = fmaf(z2, p, -0.33262279629707336f);
    p = fmaf(z2, p, 0.9999772310256958f);
    float r = z * p;
    r = big ? 1.5707963267948966f - r : r;
    return copysignf(r, t);
}

// 3D back-projection, voxel driven (the 2D one is the line kernel below):
// each thread gathers KZ3 slices of one (x, y) column from every ray of
// the subset whose Joseph taps land on them, then applies the epilogue.
// SCALED: the residual already carries each ray's scale (in-plane length
// factor times the row's cone factor), as the library's own forward
// projections write it.
template <int MODE, bool SCALED>
__global__ void __launch_bounds__(256) bp_kernel(BPArgs A)
{
    constexpr int KZ = KZ3;
    const GeoK &K = A.k;
    const unsigned nzb = (unsigned)(K.nz + KZ - 1) / KZ;     // slice blocks per image
    const int kzb = (int)(blockIdx.z % nzb);
    bp_args_at(A, blockIdx.z / nzb);
    if (MODE != BP_PLAIN && A.sc->status) return;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + ty * 32;
    const int i = blockIdx.x * 32 + tx, j = blockIdx.y * 8 + ty;
    const int kb = kzb * KZ;
    const bool inside = i < K.nx && j < K.ny;

    // detector rows (v_r, cone factor); two padding rows far outside every
    // slice carry zero weight, so a window may run up to two rows past the last
    __shared__ float2 s_row[256 + 2];
    __shared__ double s_red[4];
    for (int t = tid; t < K.nr; t += 256) s_row[t] = make_float2(A.rowv[t], A.rowf[t]);
    if (tid < 2) s_row[K.nr + tid] = make_float2(1.0e30f, 0.0f);
    __syncthreads();

    float acc[KZ];
#pragma unroll
    for (int t = 0; t < KZ; ++t) acc[t] = 0.0f;

    // block-uniform view culling (3D): rays of a view reach slices
    // zeta in z0 +- zreach * tau +- 1 for in-plane distances tau from the
    // source; with tau bounded by the block's footprint, views whose cone
    // misses the block's slices [kb, kb + KZ) are skipped
    const float bxc = fmaf((float)(blockIdx.x * 32) + 15.5f, K.dx, K.x0);
    const float byc = fmaf((float)(blockIdx.y * 8) + 3.5f, K.dy, K.y0);
    const float bhd = sqrtf(256.0f * K.dx * K.dx + 16.0f * K.dy * K.dy) + K.dmax;
    // row windows of a slice, widened by 0.01 rows for rounding
    const float rc_lo = K.row_center - 0.01f, rc_hi = K.row_center + 0.01f;
    // residual rows are gathered by 32-bit byte offsets from the subset's base
    // (the plan keeps a subset's residual below 4 GiB)
    const char *rbase = (const char *)A.r;
    const unsigned nb4 = 4u * (unsigned)K.nb;
    // the gathered row pair of a slice: r0 in [0, nr - 2] and r0 + 1 (with a
    // single detector row, row 0 twice; s_row[1] is then a padding row)
    const float r0_max = (float)max(K.nr - 2, 0);
    const unsigned row_step = K.nr > 1 ? nb4 : 0u;
    // helical subsets: z0 never decreases along the slots, so the views that
    // can reach the block's slices form one range, found by two binary
    // searches.  The bound uses tmax <= dso + |block centre| + bhd, so every
    // view left out is one the per-view test below skips as well.
    int kv_lo = 0, kv_hi = A.nview;
    if (K.z_sorted) {
        const float rmax = fmaf(K.zreach, K.dso + sqrtf(fmaf(bxc, bxc, byc * byc)) + bhd, 1.01f) + 1.0f;
        const float zlo = (float)kb - rmax, zhi = (float)(kb + KZ - 1) + rmax;
        int lo = 0, hi = A.nview;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A.views[mid].z0 < zlo) lo = mid + 1;
            else hi = mid;
        }
        kv_lo = lo;
        hi = A.nview;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A.views[mid].z0 <= zhi) lo = mid + 1;
            else hi = mid;
        }
        kv_hi = lo;
    }
    if (inside) {
        const float X = fmaf((float)i, K.dx, K.x0), Y = fmaf((float)j, K.dy, K.y0);
        const float fi = (float)i, fj = (float)j;
        for (int kv = kv_lo; kv < kv_hi; ++kv) {
            const ViewRec V = A.views[kv];
            {
                const float tmax = __builtin_amdgcn_sqrtf((bxc - V.sx) * (bxc - V.sx) + (byc - V.sy) * (byc - V.sy)) + bhd;
                const float reach = fmaf(K.zreach, tmax, 1.01f);
                if ((float)kb > V.z0 + reach || (float)(kb + KZ - 1) < V.z0 - reach) continue;
            }
            const float ddx = X - V.sx, ddy = Y - V.sy;
            const float dc = -(ddx * V.cb + ddy * V.sb);
            const float dp = ddx * V.sb - ddy * V.cb;
            const float gam = atan_window(dp * __builtin_amdgcn_rcpf(dc));   // dc > 0: in front of the source
            const float bc = fmaf(gam, K.dsd_over_ds, K.bin_center);
            const float dist = __builtin_amdgcn_sqrtf(fmaf(ddx, ddx, ddy * ddy));
            const float hw = dist > 2.0f * K.dmax ? K.dmax * __builtin_amdgcn_rcpf(dist - K.dmax) * K.dsd_over_ds + 0.05f
                                                  : (float)K.nb;
            const int b0 = max(0, (int)ceilf(bc - hw));
            const int b1 = min(K.nb - 1, (int)floorf(bc + hw));
            const RayRec *R = A.rays + (long long)kv * K.nb;
            for (int b = b0; b <= b1; ++b) {
                const RayRec rr = R[b];
                const bool ydom = meta_ydom(rr.meta);
                // the ray's in-plane interpolation weight on this column: the
                // tent 1 - |eta - o| clipped at 0
                const float fs = ydom ? fj : fi, fo = ydom ? fi : fj;
                const float eta = fmaf(fs, rr.c, rr.a);
                const float wxy = fmaxf(0.0f, 1.0f - fabsf(eta - fo));
                if (wxy == 0.0f) continue;
                {
                    const RayRecZ rz = A.raysz[(long long)kv * K.nb + b];
                    const float qz = fmaf(fs, rz.k, rz.m);
                    // detector rows per slice (it only places the row windows,
                    // which carry a 0.01-row margin)
                    const float inv = K.inv_dt * __builtin_amdgcn_rcpf(qz);
                    // row of slice coordinate k -+ 1: (k -+ 1 - z0) inv + rc
                    //   = -zk inv + (rc -+ inv), with zk = z0 - k
                    const float c_lo = rc_lo - inv, c_hi = rc_hi + inv;
                    const float base = SCALED ? wxy : wxy * rr.sc;
                    // byte offset of (view kv, row 0, channel b)
                    const unsigned cb = 4u * (unsigned)(kv * K.nr * K.nb + b);
                    // slices k >= nz (a last, partial block) are computed and
                    // dropped by the epilogue: rows are clamped, so no branch
#pragma unroll
                    for (int t = 0; t < KZ; ++t) {
                        const int k = kb + t;
                        const float zk = V.z0 - (float)k;   // zeta - k = v_r qz + zk
                        // first row r0 of the window, clamped to [0, nr - 2]
                        // so that r0 and r0 + 1 are detector rows: a row below
                        // the window's own first row lies at or beyond slice
                        // k - 1 and has weight exactly zero, so when the clamp
                        // moves r0 down the pair still sums the same terms
                        const int r0 = (int)__builtin_amdgcn_fmed3f(ceilf(fmaf(-zk, inv, c_lo)), 0.0f, r0_max);
                        const int r1 = min(K.nr - 1, (int)floorf(fmaf(-zk, inv, c_hi)));
                        // Rows r0..r1 of the window.  The linear-interpolation
                        // weight of a row at slice coordinate zeta on slice k is
                        // the tent 1 - |zeta - k| clipped at 0.  The first
                        // BP3_RW rows go without branches: weights first, their
                        // residual gathers issued together (a row of the pair
                        // outside the window lies beyond slice k -+ 1, or is a
                        // padding row, so its weight is zero and it adds an
                        // exact zero).  Row offsets: rows < 256 and 4 x channels
                        // < 2^24, so a full-rate 24-bit multiply-add.  The rows'
                        // weighted residuals are summed in row order, then
                        // scaled by the in-plane weight once.
                        static_assert(BP3_RW == 2, "the clamp of r0 keeps a pair of rows on the detector");
                        float wz[BP3_RW], rr[BP3_RW];
                        const unsigned g0 = (unsigned)__umul24((unsigned)r0, nb4) + cb;
#pragma unroll
                        for (int u = 0; u < BP3_RW; ++u) {
                            const float2 rowq = s_row[r0 + u];
                            const float w = fmaxf(0.0f, 1.0f - fabsf(fmaf(rowq.x, qz, zk)));
                            wz[u] = SCALED ? w : w * rowq.y;
                            rr[u] = *(const float *)(rbase + (g0 + (unsigned)u * row_step));
                        }
                        float sum = wz[0] * rr[0];
#pragma unroll
                        for (int u = 1; u < BP3_RW; ++u) sum = fmaf(wz[u], rr[u], sum);
                        for (int rw = r0 + BP3_RW; rw <= r1; ++rw) {
                            const float2 rowq = s_row[rw];
                            const float w1 = fmaxf(0.0f, 1.0f - fabsf(fmaf(rowq.x, qz, zk)));
                            if (w1 != 0.0f)
                                sum = fmaf(SCALED ? w1 : w1 * rowq.y,
                                           *(const float *)(rbase + ((unsigned)__umul24((unsigned)rw, nb4) + cb)), sum);
                        }
                        acc[t] = fmaf(base, sum, acc[t]);
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
                A.e.out[idx] = reg_grad_at<true>(K, A.e.x, i, j, k, A.e.beta, inv_delta2);
                part += (double)Gv * (double)Gv;
            } else {
                const float Gn = A.e.scale * acc[t];
                const float Go = A.e.G[idx], gv = A.e.g[idx];
                part += ((double)gv - (double)Gn) * ((double)Gn - (double)Go);
                A.e.g[idx] = fmaf(rho, Gn, gv) / (rho + 1.0f);
                A.e.G[idx] = Gn;
                A.e.out[idx] = reg_grad_at<true>(K, A.e.x, i, j, k, A.e.beta, inv_delta2);
            }
        }
    }
    if (MODE == BP_PLAIN) return;

    const double bsum = block_sum_256(part, s_red);
    const int blin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * kzb);
    if (tid == 0) A.partials[blin] = bsum;
}

// ------------------------------------------------------------------------
// 2D back-projection by line owners.
//
// The x-dominant rays of a view sample every image column i at
// eta = a_b + i c_b and put their two taps on rows floor(eta), floor(eta)+1 of
// that column; the y-dominant rays do the same along rows.  One launch covers
// both classes: blocks [0, nxt) own tiles of 64 columns x TR rows (a lane owns
// a column and takes the x-dominant rays), the remaining blocks own tiles of
// TR columns x 64 rows (a lane owns a row and takes the y-dominant rays).  The
// waves of a block take interleaved views.  For a view, each lane finds the
// channels whose rays cross its line inside the tile's band (channel
// coordinates of the band's two end points seen from the source); the wave
// stages the union of those rays (a, c, sc * r) in its own LDS buffers with
// coalesced loads (one array per field: the lanes of a wave read different,
// nearby rays, and single floats keep those reads off common banks), then
// every lane walks its rays in channel order and
// accumulates into its own LDS column.  No two lanes write one accumulator:
// no atomics, fixed summation order.  Waves are summed in wave order and the
// tile is written to the partial image of its class; a pointwise epilogue
// kernel adds the two partial images and applies the OS-LALM update.
constexpr int BP2_VG = 8;      // waves (view groups) per block
constexpr int BP2_TR = 16;     // band width of a tile
constexpr int BP2_LD = 64;     // LDS stride between accumulator rows: a row is one bank each per lane
constexpr int BP2_ROWS = BP2_TR + 4;   // two padding rows on each side of the band
constexpr int BP2_WMAX = 256;  // staged rays per wave and view
// the y-pass write-out transposes the tile sums through the staging arrays
static_assert(64 * (BP2_TR + 1) <= BP2_VG * BP2_WMAX, "transpose buffer exceeds the staging arrays");

// Continuous channel coordinate of the ray from the view's source through
// the point (px, py).  The point lies in front of the source (dc > 0).
__device__ inline float bin_coord(const GeoK &K, const ViewRec &V, float px, float py)
{
    const float ddx = px - V.sx, ddy = py - V.sy;
    const float dc = -(ddx * V.cb + ddy * V.sb);
    const float dp = ddx * V.sb - ddy * V.cb;
    return fmaf(atan_window(dp * __builtin_amdgcn_rcpf(dc)), K.dsd_over_ds, K.bin_center);
}

__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Accumulator slot of (row, lane) in a wave's slab.
__device__ inline int acc_slot(int row, int lane) { return row * BP2_LD + lane; }

// Two taps of one sample into the lane's accumulator column: rows fl and
// fl + 1 of the image, i.e. slab rows fl - band_base + 2 and + 3.  fl is
// clamped into [band_base - 2, band_base + TR] (rows outside the band land in
// the padding); lane_off = lane + (2 - band_base) * LD.
__device__ inline void splat2(float *slab, int lane_off, float fl, float flo, float fhi, float f, float val)
{
    const int row = (int)__builtin_amdgcn_fmed3f(fl, flo, fhi);
    float *p = slab + (row * BP2_LD + lane_off);
    p[0] += (1.0f - f) * val;
    p[BP2_LD] += f * val;
}

__global__ void __launch_bounds__(64 * BP2_VG) bp2d_lines_kernel(BPArgs A, int nxt)
{
    const GeoK &K = A.k;
    bp_args_at(A, blockIdx.y);           // image of the batch
    // a stopped run (status set) skips only the writes: every read index
    // depends on the geometry alone, so the status load need not come first
    const int status = A.sc->status;
    __shared__ float acc[BP2_VG][BP2_ROWS][BP2_LD];
    __shared__ float st_a[BP2_VG][BP2_WMAX], st_c[BP2_VG][BP2_WMAX], st_v[BP2_VG][BP2_WMAX];
    const int lane = threadIdx.x, wv = threadIdx.y;
    const int tid = lane + 64 * wv;
    for (int t = tid; t < BP2_VG * BP2_ROWS * BP2_LD; t += 64 * BP2_VG) (&acc[0][0][0])[t] = 0.0f;
    __syncthreads();

    const bool ypass = (int)blockIdx.x >= nxt;
    const int tb = ypass ? (int)blockIdx.x - nxt : (int)blockIdx.x;
    // X pass: own = column, band = rows.  Y pass: own = row, band = columns.
    const int ntx = ypass ? (K.nx + BP2_TR - 1) / BP2_TR : (K.nx + 63) / 64;
    const int own_base = (ypass ? tb / ntx : tb % ntx) * 64;
    const int band_base = (ypass ? tb % ntx : tb / ntx) * BP2_TR;
    const int n_own = ypass ? K.ny : K.nx;
    const int own = own_base + lane;
    const bool active = own < n_own;
    float *slab = &acc[wv][0][0];
    float *pa = st_a[wv], *pc = st_c[wv], *pv = st_v[wv];
    const float own_c = ypass ? fmaf((float)own, K.dy, K.y0) : fmaf((float)own, K.dx, K.x0);
    const float e1 = ypass ? fmaf((float)(band_base - 1), K.dx, K.x0) : fmaf((float)(band_base - 1), K.dy, K.y0);
    const float e2 = ypass ? fmaf((float)(band_base + BP2_TR), K.dx, K.x0)
                           : fmaf((float)(band_base + BP2_TR), K.dy, K.y0);
    const float sf = (float)own;
    const int last = min(63, n_own - 1 - own_base);   // last active lane
    const int lane_off = lane + (2 - band_base) * BP2_LD;
    const float flo = (float)(band_base - 2), fhi = (float)(band_base + BP2_TR);

    for (int kv = wv; kv < A.nview; kv += BP2_VG) {
        const ViewRec V = A.views[kv];
        const int blo = ypass ? V.by0 : V.bx0, bhi = ypass ? V.by1 : V.bx1;
        if (blo >= bhi) continue;                      // uniform across the wave
        int b0 = bhi, b1 = blo - 1;
        float u1 = 0.0f, u2 = 0.0f;
        if (active) {
            u1 = ypass ? bin_coord(K, V, e1, own_c) : bin_coord(K, V, own_c, e1);
            u2 = ypass ? bin_coord(K, V, e2, own_c) : bin_coord(K, V, own_c, e2);
            b0 = max(blo, (int)ceilf(fminf(u1, u2) - K.bin_margin));
            b1 = min(bhi - 1, (int)floorf(fmaxf(u1, u2) + K.bin_margin));
        }
        // union window of the wave: the channel coordinate over the tile's
        // band rectangle is extremal at its corners, held by the first and
        // the last active lane
        const float c1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u1), 0));
        const float c2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u2), 0));
        const float c3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u1), last));
        const float c4 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(u2), last));
        const float umin = fminf(fminf(c1, c2), fminf(c3, c4)), umax = fmaxf(fmaxf(c1, c2), fmaxf(c3, c4));
        const int wlo = max(blo, (int)ceilf(umin - K.bin_margin - 0.01f));
        const int whi = min(bhi - 1, (int)floorf(umax + K.bin_margin + 0.01f));
        if (whi < wlo) continue;
        b0 = max(b0, wlo);                             // keep every lane inside the union
        b1 = min(b1, whi);
        const RayRec *R = A.rays + (long long)kv * K.nb;
        const float *rv = A.r + (long long)kv * K.nb;
        if (whi - wlo + 1 <= BP2_WMAX) {
            wave_lds_sync();                           // previous view's readers are done
            for (int t = lane; t <= whi - wlo; t += 64) {
                const RayRec q = R[wlo + t];
                pa[t] = q.a;
                pc[t] = q.c;
                pv[t] = q.sc * rv[wlo + t];
            }
            wave_lds_sync();
            // lanes whose window lies outside the union never happen (the
            // union covers every lane), so index b - wlo stays in range
            int b = b0;
            for (; b + 3 <= b1; b += 4) {
                float qa[4], qc[4], qv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    qa[u] = pa[b + u - wlo];
                    qc[u] = pc[b + u - wlo];
                    qv[u] = pv[b + u - wlo];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float eta = fmaf(sf, qc[u], qa[u]);
                    const float fl = floorf(eta);
                    splat2(slab, lane_off, fl, flo, fhi, eta - fl, qv[u]);
                }
            }
            for (; b <= b1; ++b) {
                const float eta0 = fmaf(sf, pc[b - wlo], pa[b - wlo]);
                const float fl0 = floorf(eta0);
                splat2(slab, lane_off, fl0, flo, fhi, eta0 - fl0, pv[b - wlo]);
            }
        } else {
            for (int b = b0; b <= b1; ++b) {           // wide window: read rays directly
                const RayRec q = R[b];
                const float eta = fmaf(sf, q.c, q.a);
                const float fl = floorf(eta);
                splat2(slab, lane_off, fl, flo, fhi, eta - fl, q.sc * rv[b]);
            }
        }
    }
    __syncthreads();
    if (A.check_status && status) return;

    // sum the waves in order and write the tile to its class's partial image;
    // consecutive threads walk along x in global memory
    if (!ypass) {
        for (int t = tid; t < BP2_TR * 64; t += 64 * BP2_VG) {
            const int bnd = t / 64, ow = t % 64;
            const int i = own_base + ow, j = band_base + bnd;
            if (i >= K.nx || j >= K.ny) continue;
            const int slot = acc_slot(bnd + 2, ow);
            float sacc = (&acc[0][0][0])[slot];
#pragma unroll
            for (int w2 = 1; w2 < BP2_VG; ++w2) sacc += (&acc[w2][0][0])[slot];
            A.part[(long long)j * K.nx + i] = sacc;
        }
        return;
    }
    // y pass: x runs along the band, i.e. across accumulator rows, so the
    // waves are summed with the lane (own) index fastest and the sums go
    // through a transpose with a row stride of TR + 1 (the staging arrays are
    // free by now), which keeps both LDS passes off common banks
    float *tr = &st_a[0][0];
    for (int t = tid; t < BP2_TR * 64; t += 64 * BP2_VG) {
        const int bnd = t / 64, ow = t % 64;
        const int slot = acc_slot(bnd + 2, ow);
        float sacc = (&acc[0][0][0])[slot];
#pragma unroll
        for (int w2 = 1; w2 < BP2_VG; ++w2) sacc += (&acc[w2][0][0])[slot];
        tr[ow * (BP2_TR + 1) + bnd] = sacc;
    }
    __syncthreads();
    for (int t = tid; t < BP2_TR * 64; t += 64 * BP2_VG) {
        const int bnd = t % BP2_TR, ow = t / BP2_TR;
        const int i = band_base + bnd, j = own_base + ow;
        if (i >= K.nx || j >= K.ny) continue;
        A.part2[(long long)j * K.nx + i] = tr[ow * (BP2_TR + 1) + bnd];
    }
}

// Pointwise epilogue of the 2D back-projection: total = part_x + part_y, then
// PLAIN (out = scale * total, or +=) or INIT as in the 3D kernel (STEP is
// the step kernel below).
template <int MODE>
__global__ void __launch_bounds__(256) bp2d_epilogue_kernel(BPArgs A)
{
    const GeoK &K = A.k;
    bp_args_at(A, blockIdx.z);           // image of the batch
    if (MODE != BP_PLAIN && A.sc->status) return;
    __shared__ double s_red[4];
    const int tid = threadIdx.x + 32 * threadIdx.y;
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y;
    double part = 0.0;
    if (i < K.nx && j < K.ny) {
        const long long idx = (long long)j * K.nx + i;
        const float total = A.part[idx] + A.part2[idx];
        if (MODE == BP_PLAIN) {
            const float vv = A.e.scale * total;
            A.e.out[idx] = A.e.accumulate ? A.e.out[idx] + vv : vv;
        } else {
            const float Gv = A.e.scale * total;
            A.e.G[idx] = Gv;
            A.e.g[idx] = Gv;
            A.e.out[idx] = reg_grad_at<false>(K, A.e.x, i, j, 0, A.e.beta, A.e.inv_delta2);
            part = (double)Gv * (double)Gv;
        }
    }
    if (MODE == BP_PLAIN) return;
    const double bsum = block_sum_256(part, s_red);
    const int blin = blockIdx.x + gridDim.x * blockIdx.y;
    if (threadIdx.x + 32 * threadIdx.y == 0) A.partials[blin] = bsum;
}

// 2D step epilogue, fused with the next step's x-update (one thread per
// pixel of a 32x32 tile).  G+ = M (part + part2); the restart-indicator
// partial (g - G+)(G+ - G) in FP64; g <- (rho G+ + g) / (rho + 1); G <- G+.
// x of this step is xs[sel].  Not LAST: the next step's x for each value
// its rho can take once the pending decision is made (candidate 0: restart,
// rho_0 = 1, or the fixed rho; candidate 1: continue, rho_{l+1}), written
// to xo and to the layout set of the candidate (XN directly, XT through an
// LDS transpose).  LAST: grad R(x) instead, as the plain epilogue.  Block
// partial: wave butterflies, then the 16 wave sums in order.
struct Step2dArgs {
    GeoK k;
    const float *part, *part2;
    float *G, *g;
    const float *xs0, *xs1;
    float *xw;
    const float *denom;
    float *gradR;
    float *xo0, *xo1, *XT0, *XN0, *XT1, *XN1;
    const DevScalars *sc;
    double *partials;
    float scale, beta, inv_delta2;
    double rho_min;
    int continuation, nonneg;
    int tiles_x, tiles_y;   // 32 x 32 tiles; partial of tile (bx, by) at bx + tiles_x by
    BatchStr bs;            // image b = blockIdx.z
};

template <bool LAST>
__global__ void __launch_bounds__(1024) step2d_kernel(Step2dArgs A)
{
    const GeoK &K = A.k;
    __shared__ float tile[2][32][33];
    __shared__ float nbr[34][35];          // x of this step over the tile and a one-pixel halo
    __shared__ double s_red[16];
    __shared__ float s_rho1;
    {
        // image bi of the batch
        const long long bi = blockIdx.z, im = bi * A.bs.img;
        A.part += im;
        A.part2 += im;
        A.G += im;
        A.g += im;
        A.xs0 += im;
        A.xs1 += im;
        if (A.xw) A.xw += im;
        if (A.denom) A.denom += im;
        A.gradR += im;
        if (A.xo0) A.xo0 += im;
        if (A.xo1) A.xo1 += im;
        if (A.XT0) A.XT0 += bi * A.bs.layT;
        if (A.XN0) A.XN0 += bi * A.bs.layN;
        if (A.XT1) A.XT1 += bi * A.bs.layT;
        if (A.XN1) A.XN1 += bi * A.bs.layN;
        A.sc += bi;
        A.partials += bi * A.bs.part;
    }
    // tile of this block: the hardware hands consecutive blocks to the eight
    // XCDs in turn; XCD c takes the c-th eighth of the tiles in column-major
    // order (a strip of whole tile columns), so the left and right halo
    // lines of the neighbourhood loads are shared inside one XCD's L2.  The
    // grid is padded to a multiple of 8; padding blocks have no tile.
    const int ntile = A.tiles_x * A.tiles_y;
    const int tl = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
    if (tl >= ntile) return;
    const int bx = tl / A.tiles_y, by = tl - bx * A.tiles_y;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + 32 * ty;
    const int i0 = bx * 32, j0 = by * 32;
    const int i = i0 + tx, j = j0 + ty;
    const bool inside = i < K.nx && j < K.ny;
    const long long idx = (long long)j * K.nx + i;
    // the scalar record and the loads that do not depend on it go out
    // together, before its status is tested (threads outside the image read
    // pixel 0; pixel indices are clamped into the image)
    const DevScalars s = *A.sc;
    const long long ldx = inside ? idx : 0;
    const float p0 = A.part[ldx], p1 = A.part2[ldx], Go = A.G[ldx], gv = A.g[ldx];
    const float dv = LAST ? 0.0f : A.denom[ldx];
    // x at this pixel and at one pixel of the tile's halo (threads 0..131:
    // the rows above and below, then the columns left and right), for both
    // candidates: the record's choice is not known yet
    const long long cdx = (long long)min(j, K.ny - 1) * K.nx + min(i, K.nx - 1);
    const float c0 = A.xs0[cdx], c1 = A.xs1[cdx];
    const bool halo = tid < 132;
    const int hy = tid < 34 ? -1 : (tid < 68 ? 32 : (tid < 100 ? tid - 68 : tid - 100));
    const int hx = tid < 34 ? tid - 1 : (tid < 68 ? tid - 35 : (tid < 100 ? -1 : 32));
    float h0 = 0.0f, h1 = 0.0f;
    if (halo) {
        const long long hdx = (long long)min(max(j0 + hy, 0), K.ny - 1) * K.nx + min(max(i0 + hx, 0), K.nx - 1);
        h0 = A.xs0[hdx];
        h1 = A.xs1[hdx];
    }
    // keeps the compiler from sinking those loads below the status test
    asm volatile("" ::: "memory");
    if (s.status) return;
    const bool sel = s.sel != 0;
    nbr[ty + 1][tx + 1] = sel ? c1 : c0;
    if (halo) nbr[hy + 1][hx + 1] = sel ? h1 : h0;
    const float rho = (float)s.rho;
    const bool two = A.continuation != 0;
    // rho of the continuing candidate, once per block
    if (!LAST && two && tid == 0) s_rho1 = (float)continuation_rho(s.l + 1, A.rho_min);
    // the pointwise part while the neighbourhood is being staged
    double part = 0.0;
    float Gn = 0.0f, gn = 0.0f;
    if (inside) {
        Gn = A.scale * (p0 + p1);
        part = ((double)gv - (double)Gn) * ((double)Gn - (double)Go);
        gn = fmaf(rho, Gn, gv) / (rho + 1.0f);
        A.G[idx] = Gn;
        A.g[idx] = gn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = part;
    __syncthreads();
    Nbr2d nx;
#pragma unroll
    for (int t = 0; t < 9; ++t) nx.v[t] = nbr[ty + t / 3][tx + t % 3];
    float v0 = 0.0f, v1 = 0.0f;
    if (inside) {
        // a tile whose halo lies inside the image drops no neighbour
        const bool interior = i0 >= 1 && j0 >= 1 && i0 + 33 <= K.nx && j0 + 33 <= K.ny;
        const float rv = interior ? reg_grad_2d_inner(nx, A.beta, A.inv_delta2)
                                  : reg_grad_2d(K, nx, i, j, A.beta, A.inv_delta2);
        const float xv = nx.v[4];
        if (A.xw) A.xw[idx] = xv;
        if (LAST) {
            A.gradR[idx] = rv;
        } else {
            const float curv = A.beta * reg_curv_sum(K, i, j, 0);
            const float alpha = (float)s.alpha;
            const long long n_idx = (long long)j * K.ldN + i + 2;
            v0 = x_update(xv, Gn, gn, rv, two ? 1.0f : rho, alpha, dv, curv, A.nonneg);
            A.xo0[idx] = v0;
            A.XN0[n_idx] = v0;
            if (two) {
                v1 = x_update(xv, Gn, gn, rv, s_rho1, alpha, dv, curv, A.nonneg);
                A.xo1[idx] = v1;
                A.XN1[n_idx] = v1;
            }
        }
    }
    if (tid == 0) {
        double t = s_red[0];
#pragma unroll
        for (int w = 1; w < 16; ++w) t += s_red[w];
        A.partials[bx + A.tiles_x * by] = t;
    }
    if (LAST) return;
    tile[0][ty][tx] = v0;
    tile[1][ty][tx] = v1;
    __syncthreads();
    const int it = i0 + ty, jt = j0 + tx;
    if (it < K.nx && jt < K.ny) {
        const long long t_idx = (long long)it * K.ldT + jt + 2;
        A.XT0[t_idx] = tile[0][tx][ty];
        if (two) A.XT1[t_idx] = tile[1][tx][ty];
    }
}

// One block: fixed-order FP64 sum of the back-projection's block partials,
// then the continuation decision (STEP) or the finite check (INIT); reads
// the scalar record `in`, writes the next one to `out`.
// WAVE (2D): the one-wave fixed order that the fused decisions of the
// x-update and forward-projection kernels use, so a decision gives the same
// bits wherever it is taken.
template <int MODE, bool WAVE>
__global__ void __launch_bounds__(256) finalize_kernel(const double *partials, long long nblocks,
                                                       const DevScalars *in, DevScalars *out, ContArgs C,
                                                       long long part_stride)
{
    __shared__ double s_w[4];
    const int tid = threadIdx.x;
    // one block per image of the batch
    partials += (long long)blockIdx.x * part_stride;
    in += blockIdx.x;
    out += blockIdx.x;
    C = cont_at(C, (int)blockIdx.x);
    const DevScalars s = *in;
    if (s.status) {
        if (tid == 0) *out = s;
        return;
    }
    const double total = WAVE ? fixed_sum_wave(partials, nblocks, tid & 63) : fixed_sum_256(partials, nblocks, tid, s_w);
    if (tid == 0) *out = continuation_update(s, C, total, MODE == BP_INIT, true);
}

template <bool SCALED>
hipError_t bp_dispatch_scaled(const lalm_plan *p, const BPArgs &a, int mode, dim3 grd, hipStream_t st)
{
    dim3 blk(32, 8);
    if (mode == BP_PLAIN) return klaunch(p, bp_kernel<BP_PLAIN, SCALED>, grd, blk, st, a);
    if (mode == BP_INIT) return klaunch(p, bp_kernel<BP_INIT, SCALED>, grd, blk, st, a);
    return klaunch(p, bp_kernel<BP_STEP, SCALED>, grd, blk, st, a);
}

hipError_t bp_dispatch(const lalm_plan *p, const BPArgs &a, int mode, dim3 grd, hipStream_t st)
{
    return a.e.ray_scaled ? bp_dispatch_scaled<true>(p, a, mode, grd, st)
                          : bp_dispatch_scaled<false>(p, a, mode, grd, st);
}

template <bool IS3D>
__global__ void __launch_bounds__(256) reg_grad_kernel(GeoK K, const float *x, float *out, float beta,
                                                       float inv_delta2)
{
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y;
    const int k = (int)(blockIdx.z % (unsigned)K.nz);
    const long long im = (long long)(blockIdx.z / (unsigned)K.nz) * ((long long)K.nx * K.ny * K.nz);
    x += im;                               // image of the batch
    out += im;
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
    a.sc = cur_sc(p);
    a.part = p->d_part;
    a.part2 = p->d_part2;
    a.check_status = mode != BP_PLAIN;
    a.bs = batch_str(p);
    if (!p->is3d) {
        const int nxt = ((p->nx + 63) / 64) * ((p->ny + BP2_TR - 1) / BP2_TR);
        const int nyt = ((p->nx + BP2_TR - 1) / BP2_TR) * ((p->ny + 63) / 64);
        const hipError_t el = klaunch(p, bp2d_lines_kernel, dim3(nxt + nyt, p->B), dim3(64, BP2_VG), st, a, nxt);
        if (el != hipSuccess || mode == BP_LINES) return el;
        if (mode == BP_STEP) return launch_step2d(p, e.x, e.x, nullptr, nullptr, nullptr, e, nullptr, 0, true, st);
        dim3 ge((p->nx + 31) / 32, (p->ny + 7) / 8, p->B);
        a.nblocks = (int)(ge.x * ge.y);
        if (mode == BP_PLAIN) hipLaunchKernelGGL((bp2d_epilogue_kernel<BP_PLAIN>), ge, dim3(32, 8), 0, st, a);
        else hipLaunchKernelGGL((bp2d_epilogue_kernel<BP_INIT>), ge, dim3(32, 8), 0, st, a);
    } else {
        if (mode == BP_LINES) return hipErrorInvalidValue;
        const int kz = KZ3;
        const unsigned nzb = (unsigned)(p->nz + kz - 1) / kz;
        dim3 grd((p->nx + 31) / 32, (p->ny + 7) / 8, nzb * p->B);
        a.nblocks = (int)(grd.x * grd.y * nzb);
        hipError_t e = bp_dispatch(p, a, mode, grd, st);
        if (e != hipSuccess) return e;
    }
    if (mode == BP_PLAIN) return hipGetLastError();
    p->bp_nblocks = a.nblocks;
    if (mode == BP_INIT) {
        // finite check of the initial gradient: scalars advance to the other record
        if (p->is3d)
            hipLaunchKernelGGL((finalize_kernel<BP_INIT, false>), dim3(p->B), dim3(256), 0, st,
                               (const double *)p->d_partials, p->bp_nblocks, (const DevScalars *)cur_sc(p),
                               nxt_sc(p), e.cont, (long long)p->n_partials);
        else
            hipLaunchKernelGGL((finalize_kernel<BP_INIT, true>), dim3(p->B), dim3(256), 0, st,
                               (const double *)p->d_partials, p->bp_nblocks, (const DevScalars *)cur_sc(p),
                               nxt_sc(p), e.cont, (long long)p->n_partials);
        p->sc_cur ^= 1;
    }
    return hipGetLastError();
}

hipError_t launch_step2d(const lalm_plan *p, const float *xs0, const float *xs1, float *xw, float *xo0,
                         float *xo1, const BpEpi &e, const float *denom, int nonneg, bool last, hipStream_t st)
{
    if (p->is3d) return hipErrorInvalidValue;
    if (!last && (!xo0 || !xo1 || !denom || !p->d_xt1 || !p->d_xn1)) return hipErrorInvalidValue;
    Step2dArgs a;
    a.k = p->k;
    a.part = p->d_part;
    a.part2 = p->d_part2;
    a.G = e.G;
    a.g = e.g;
    a.xs0 = xs0;
    a.xs1 = xs1;
    a.xw = xw;
    a.denom = denom;
    a.gradR = p->d_gradR;
    a.xo0 = xo0;
    a.xo1 = xo1;
    a.XT0 = p->d_xt;
    a.XN0 = p->d_xn;
    a.XT1 = p->d_xt1;
    a.XN1 = p->d_xn1;
    a.sc = cur_sc(p);
    a.partials = p->d_partials;
    a.scale = e.scale;
    a.beta = e.beta;
    a.inv_delta2 = e.inv_delta2;
    a.rho_min = e.cont.rho_min;
    a.continuation = e.cont.continuation;
    a.nonneg = nonneg;
    a.bs = batch_str(p);
    a.tiles_x = (p->nx + 31) / 32;
    a.tiles_y = (p->ny + 31) / 32;
    const int ntile = a.tiles_x * a.tiles_y;
    const dim3 grd((unsigned)((ntile + 7) / 8 * 8), 1, p->B);   // padded to the eight XCDs
    p->bp_nblocks = ntile;
    return last ? klaunch(p, step2d_kernel<true>, grd, dim3(32, 32), st, a)
                : klaunch(p, step2d_kernel<false>, grd, dim3(32, 32), st, a);
}

hipError_t launch_finalize(const lalm_plan *p, const ContArgs &c, hipStream_t st)
{
    const double *part = p->d_partials;
    const DevScalars *in = cur_sc(p);
    DevScalars *out = nxt_sc(p);
    const long long ps = p->n_partials;
    const dim3 g(p->B);
    const hipError_t e = p->is3d
        ? klaunch(p, finalize_kernel<BP_STEP, false>, g, dim3(256), st, part, p->bp_nblocks, in, out, c, ps)
        : klaunch(p, finalize_kernel<BP_STEP, true>, g, dim3(256), st, part, p->bp_nblocks, in, out, c, ps);
    p->sc_cur ^= 1;
    return e;
}

hipError_t launch_reg_grad(const lalm_plan *p, const float *x, float beta, float inv_delta2,
                           hipStream_t st)
{
    dim3 blk(32, 8), grd((p->nx + 31) / 32, (p->ny + 7) / 8, (unsigned)(p->nz * p->B));
    if (p->is3d)
        hipLaunchKernelGGL((reg_grad_kernel<true>), grd, blk, 0, st, p->k, x, p->d_gradR, beta, inv_delta2);
    else
        hipLaunchKernelGGL((reg_grad_kernel<false>), grd, blk, 0, st, p->k, x, p->d_gradR, beta, inv_delta2);
    return hipGetLastError();
}

}  // namespace lalm
