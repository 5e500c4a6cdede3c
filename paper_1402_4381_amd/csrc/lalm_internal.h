// Internal declarations of the gfx950 OS-LALM library (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lalm.h"

namespace lalm {

// ---------------------------------------------------------------- tables
//
// Per (sinogram slot, bin) Joseph parameters, computed in FP64 on the host
// and stored as FP32.  For slice s of the dominant in-plane axis the sample
// sits at fractional index eta(s) = a + s*c along the other in-plane axis;
// sc is the in-plane ray length per slice.  meta packs the dominant axis
// (bit 31: 0 = x, 1 = y) and the conservative slice range [s_lo, s_hi]
// (bits 0..15 and 16..30) outside of which no tap can fall inside the image.
struct RayRec {
    float a, c, sc;
    uint32_t meta;
};
// 3D only: q(s) = m + s*k; the slice coordinate of the sample is
// zeta = z0(view) + v_r * q(s).
struct RayRecZ {
    float m, k;
};
// Per slot: source position (mm, relative to the isocentre), cos/sin of the
// view angle, z0 = (S_z - Z_0) / dz, and the channel ranges [bx0, bx1) and
// [by0, by1) of the view's x-dominant and y-dominant rays (each class is one
// contiguous range because the fan is narrower than 90 degrees).
struct ViewRec {
    float sx, sy, cb, sb;
    float z0, pad0;
    int bx0, bx1, by0, by1;
    int pad1, pad2;
};

constexpr uint32_t kYDom = 0x80000000u;
__host__ __device__ inline int meta_lo(uint32_t m) { return int(m & 0xFFFFu); }
__host__ __device__ inline int meta_hi(uint32_t m) { return int((m >> 16) & 0x7FFFu); }
__host__ __device__ inline bool meta_ydom(uint32_t m) { return (m & kYDom) != 0; }

// Scalars that live on the device across the steps of lalm_iterate.
struct DevScalars {
    double rho;       // rho used by the next step
    double xi;        // last restart indicator
    long long l;      // continuation counter
    long long step;   // global subset-step counter
    int status;       // 0 ok, 1 non-finite restart indicator met
    int sel;          // 2D fused steps: x-update candidate the last decision
                      // selected (0: restart or fixed rho, 1: continue)
    double alpha;     // Barzilai-Borwein scale of D_L (1 without it)
};

// Element strides of a batch of images planned together (elements of
// float or double): an image, one XT / XN layout, the reduction partials of
// one image.  Kernels add b times these to their pointers for image b.
struct BatchStr {
    long long img, layT, layN, part;
};

// Geometry constants handed to kernels by value.
struct GeoK {
    int nx, ny, nz, nb, nr;
    int is3d;
    float dx, dy, dz;
    float x0, y0;             // centre of voxel (0, 0) in mm
    float dsd_over_ds;        // bins per radian of fan angle
    float bin_center;         // (nb-1)/2 + channel offset
    float dmax;               // max(dx, dy)
    float inv_dt;             // 1 / dt
    float row_center;         // (nr-1)/2
    float bin_margin;         // channel-window margin (bins) for rounding and the window atan
    float zreach;             // 3D: ((nr-1)/2 dt) / (dsd dz), slices reached per mm of in-plane path
    float dso;                // source to isocentre (mm)
    int z_sorted;             // 3D: z0 never decreases along the slots of a subset (helical)
    // padded image copies
    int ldT, ldN;             // padded length of the fastest axis: ny+4, nx+4
    long long slabT, slabN;   // elements per slice of the dominant axis
};

// Continuation bookkeeping (restart rule, rho schedule, statistics).  With
// a batch, element b's forced bits start at forced + b forced_len and its
// statistics at st_* + b st_cap.
struct ContArgs {
    int continuation;
    double rho_fixed, rho_min;
    const uint8_t *forced;
    long long forced_len;
    double *st_rho, *st_xi;
    uint8_t *st_restart;
    long long st_cap;
};

// Element b of a batch: the forced bits and statistics of that image.
__host__ __device__ inline ContArgs cont_at(ContArgs c, int b)
{
    if (c.forced) c.forced += (long long)b * c.forced_len;
    if (c.st_rho) c.st_rho += (long long)b * c.st_cap;
    if (c.st_xi) c.st_xi += (long long)b * c.st_cap;
    if (c.st_restart) c.st_restart += (long long)b * c.st_cap;
    return c;
}

// Fixed-order FP64 sum of v[0..n): thread t < 256 adds v[t], v[t+256], ...
// in turn, each of the four waves combines its lanes by an xor butterfly,
// then (w0 + w1) + (w2 + w3).  Every block that calls it gets the same bits.
// All threads of the block must call it (tid = linear thread index, blocks
// of >= 256 threads, wave64); s_w holds 4 doubles of LDS.
__device__ inline double fixed_sum_256(const double *v, long long n, int tid, double *s_w)
{
    double a = 0.0;
    if (tid < 256) {
        long long t = tid;
        // loads in batches (one memory round trip each), additions in order
        for (; t + 7 * 256 < n; t += 8 * 256) {
            double u[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) u[k] = v[t + k * 256];
#pragma unroll
            for (int k = 0; k < 8; ++k) a += u[k];
        }
        for (; t < n; t += 256) a += v[t];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (tid < 256 && (tid & 63) == 0) s_w[tid >> 6] = a;
    __syncthreads();
    const double r = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
    __syncthreads();
    return r;
}

// Fixed-order FP64 sum of v[0..n) within one wave: lane t adds v[t],
// v[t+64], ... in turn, then an xor butterfly over the lanes.  Floating-point
// addition is commutative, so every lane of every wave that calls it holds
// the same bits: the waves of many blocks can each take the same decision
// from it without a barrier.  lane = lane index in the wave64.
__device__ inline double fixed_sum_wave(const double *v, long long n, int lane)
{
    double a = 0.0;
    long long t = lane;
    // loads in batches (one memory round trip each), additions in order
    for (; t + 7 * 64 < n; t += 8 * 64) {
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = v[t + k * 64];
#pragma unroll
        for (int k = 0; k < 8; ++k) a += u[k];
    }
    if (t + 3 * 64 < n) {
        double u[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) u[k] = v[t + k * 64];
#pragma unroll
        for (int k = 0; k < 4; ++k) a += u[k];
        t += 4 * 64;
    }
    for (; t < n; t += 64) a += v[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// d psi / dt for the hyperbola potential: t / sqrt(1 + (t/delta)^2).  The
// argument of the reciprocal square root is at least 1, so the hardware
// instruction alone gives what rsqrtf gives (rsqrtf adds a rescaling for
// denormal arguments around the same instruction).
__device__ inline float dpsi(float t, float inv_delta2)
{
    return t * __builtin_amdgcn_rsqf(fmaf(t * t, inv_delta2, 1.0f));
}

// grad R at voxel (i, j, k): beta sum_{n in N} kappa psi'(x_c - x_n)
template <bool IS3D>
__device__ inline float reg_grad_at(const GeoK &K, const float *x, int i, int j, int k, float beta,
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

// 2D: the 3x3 neighbourhood of pixel (i, j), loaded with indices clamped
// into the image (every load is in bounds; neighbours outside are dropped by
// reg_grad_2d), so the loads can be issued before it is known which image
// they will serve.  v[4] is the centre; v[3 (dy + 1) + (dx + 1)].
struct Nbr2d {
    float v[9];
};
__device__ inline Nbr2d load_nbr2d(const GeoK &K, const float *x, int i, int j)
{
    Nbr2d n;
    const int ic = min(max(i, 0), K.nx - 1), jc = min(max(j, 0), K.ny - 1);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int jj = min(max(jc + dy, 0), K.ny - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int ii = min(max(ic + dx, 0), K.nx - 1);
            n.v[3 * (dy + 1) + (dx + 1)] = x[(long long)jj * K.nx + ii];
        }
    }
    return n;
}
// reg_grad_at<false> from a loaded neighbourhood: the same terms in the same
// order, so the result is bit-identical.
__device__ inline float reg_grad_2d(const GeoK &K, const Nbr2d &n, int i, int j, float beta, float inv_delta2)
{
    const float r2 = 0.70710678118654752f;
    const float xc = n.v[4];
    float s = 0.0f;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int ii = i + dx, jj = j + dy;
            const bool in = ii >= 0 && ii < K.nx && jj >= 0 && jj < K.ny;
            const float kap = (dx != 0 && dy != 0) ? r2 : 1.0f;
            const float t = fmaf(kap, dpsi(xc - n.v[3 * (dy + 1) + (dx + 1)], inv_delta2), s);
            s = in ? t : s;
        }
    }
    return beta * s;
}
// reg_grad_2d for a pixel whose eight neighbours all lie inside the image:
// the same terms in the same order, without the bounds tests.
__device__ inline float reg_grad_2d_inner(const Nbr2d &n, float beta, float inv_delta2)
{
    const float r2 = 0.70710678118654752f;
    const float xc = n.v[4];
    float s = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        if (t == 4) continue;
        const float kap = (t == 0 || t == 2 || t == 6 || t == 8) ? r2 : 1.0f;
        s = fmaf(kap, dpsi(xc - n.v[t], inv_delta2), s);
    }
    return beta * s;
}

// Number-weighted neighbour sum 2 * sum_{k in N(j)} kappa_jk for voxel (i,j,k)
// (the separable majorizer curvature of the hyperbola regularizer over beta).
__device__ inline float reg_curv_sum(const GeoK &K, int i, int j, int k)
{
    const float r2 = 0.70710678118654752f, r3 = 0.57735026918962576f;
    int cx = (i > 0) + (i < K.nx - 1);
    int cy = (j > 0) + (j < K.ny - 1);
    int cz = K.is3d ? (k > 0) + (k < K.nz - 1) : 0;
    // neighbours along 1, 2 or 3 axes: counts are products of per-axis counts
    float s1 = (float)(cx + cy + cz);
    float s2 = (float)(cx * cy + cx * cz + cy * cz);
    float s3 = (float)(cx * cy * cz);
    return 2.0f * (s1 + s2 * r2 + s3 * r3);
}

// The n = 1 x-update of a step (one projected gradient step on the inner
// problem, Sec. IV-A): s = rho G + (1 - rho) g, then
// x+ = max(0, x - (s + grad R(x)) / (rho alpha D_L + beta C)) where
// beta C = curv_b is the regularizer's separable curvature; a pixel with a
// zero denominator keeps its value.  Every kernel that updates x calls this,
// so all paths give the same bits.
__device__ inline float x_update(float x, float G, float g, float gR, float rho, float alpha, float dl,
                                 float curv_b, int nonneg)
{
    const float num = fmaf(rho, G, (1.0f - rho) * g) + gR;
    const float den = fmaf(rho * alpha, dl, curv_b);
    float v = x;
    if (den > 0.0f) {
        v = v - num / den;
        if (nonneg) v = fmaxf(v, 0.0f);
    }
    return v;
}

// rho_l of the downward continuation (eq. rho_l_formula_qp): 1 at l = 0,
// else (pi/(l+1)) sqrt(1 - (pi/(2(l+1)))^2), never below rho_min.
__device__ inline double continuation_rho(long long l, double rho_min)
{
    if (l == 0) return 1.0;
    const double pi = 3.14159265358979323846;
    const double a = pi / (2.0 * (double)(l + 1));
    return fmax(pi / (double)(l + 1) * sqrt(1.0 - a * a), rho_min);
}

// Decision after the back-projection of step in.step, from its restart
// indicator xi (Sec. III-B: restart, i.e. l = 0, when xi > 0): returns the
// scalars of the next step.  init: after the initial gradient, only the
// finite check.  record: write the step's statistics (one thread only).
__device__ inline DevScalars continuation_update(const DevScalars &in, const ContArgs &C, double xi, bool init,
                                                 bool record)
{
    DevScalars o = in;
    if (init) {
        if (!isfinite(xi)) o.status = 1;
        return o;
    }
    const long long jstep = in.step;
    bool restart = false;
    if (!isfinite(xi)) {
        o.status = 1;
    } else if (C.continuation) {
        restart = xi > 0.0;
        if (C.forced && jstep < C.forced_len) restart = C.forced[jstep] != 0;
        o.l = restart ? 0 : in.l + 1;
        o.rho = continuation_rho(o.l, C.rho_min);
    }
    if (!o.status) o.sel = (C.continuation && o.l != 0) ? 1 : 0;
    o.xi = xi;
    if (record && jstep < C.st_cap) {
        if (C.st_rho) C.st_rho[jstep] = in.rho;
        if (C.st_xi) C.st_xi[jstep] = xi;
        if (C.st_restart) C.st_restart[jstep] = restart ? 1 : 0;
    }
    o.step = jstep + 1;
    return o;
}

}  // namespace lalm

struct lalm_plan {
    lalm_geometry g;
    int M = 0;
    // images planned together: every image-sized buffer (the caller's and
    // the plan's workspace) holds B images of nvox voxels one after the
    // other, every sinogram-sized one B sinograms, and each kernel launch
    // covers all B
    int B = 1;
    int64_t nvox = 0;
    int64_t layT = 0, layN = 0;         // elements of one image's XT / XN layout
    int nx = 0, ny = 0, nz = 0, nb = 0, nr = 0, nv = 0;
    bool is3d = false;
    int device = 0;
    std::vector<int32_t> order;
    std::vector<int32_t> view_of_slot;
    std::vector<int64_t> slot_offset;   // [M+1] first slot of each subset
    std::vector<int64_t> subset_samples;
    int64_t rays_per_view = 0;
    int64_t max_subset_rays = 0;
    lalm::GeoK k{};
    // device memory owned by the plan
    lalm::RayRec *d_rays = nullptr;     // [n_views][nb] in slot order
    lalm::RayRecZ *d_raysz = nullptr;   // [n_views][nb] (3D)
    lalm::ViewRec *d_views = nullptr;   // [n_views] in slot order
    float *d_rowv = nullptr;            // [nr] v_r (mm)
    float *d_rowf = nullptr;            // [nr] sqrt(1 + (v_r/dsd)^2)
    float *d_xt = nullptr;              // padded copy for x-dominant rays
    float *d_xn = nullptr;              // padded copy for y-dominant rays
    float *d_gradR = nullptr;           // regularizer gradient image
    float *d_r = nullptr;               // subset residual
    float *d_part = nullptr;            // 2D: back-projection of the x-dominant rays
    float *d_part2 = nullptr;           // 2D: back-projection of the y-dominant rays
    float *d_v = nullptr;               // inner FISTA iterate (n_inner > 1); part, part2 hold z
    float *d_fbpq = nullptr;            // 2D: filtered sinogram of the FBP
    // 2D fused steps: the second set of projector layouts and the x-update
    // candidates of two consecutive steps ([2 steps][2 candidates][image])
    float *d_xt1 = nullptr, *d_xn1 = nullptr;
    float *d_xc = nullptr;
    double *d_partials = nullptr;       // reduction partials, n_partials per image
    int64_t n_partials = 0;
    // two device scalar records: each continuation decision reads one and
    // writes the other (kernels of a launch that make the decision
    // redundantly per block never see a half-updated record); sc_cur is the
    // host's index of the current one, advanced in launch order
    lalm::DevScalars *d_sc = nullptr;   // [2][B]
    mutable int sc_cur = 0;
    mutable long long bp_nblocks = 0;   // partials (per image) written by the last STEP back-projection
    lalm::DevScalars *h_sc = nullptr;   // pinned host mirror [B]
    double *d_tmp = nullptr;            // small FP64 scratch (monitors), 64 + M per image
    int fp_nseg = 1;
    // optional per-kernel event timing
    // (each timed kernel carries its own start / stop events on its dispatch;
    // a class is the set of kernels of one part of a step)
    bool prof = false;
    mutable std::vector<hipEvent_t> prof_ev;   // pool: pairs (start, stop)
    mutable std::vector<int> prof_kind;        // class of each recorded pair
    mutable size_t prof_used = 0;
    mutable int prof_cls = -1;                 // class being recorded, -1: none
    double prof_ms[3] = {0, 0, 0};
    int64_t prof_n[3] = {0, 0, 0};             // class instances (steps)
};

namespace lalm {

void set_error(const std::string &msg);

// With profiling on and a class open: a (start, stop) event pair for one
// kernel launch, attributed to that class.
bool prof_pair(const lalm_plan *p, hipEvent_t *start, hipEvent_t *stop);

// Kernel launch that, while profiling, times the kernel by the events of
// its own dispatch (no extra packets in the stream between kernels).
template <typename K, typename... Args>
inline hipError_t klaunch(const lalm_plan *p, K kernel, dim3 grid, dim3 block, hipStream_t st, Args... args)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof_pair(p, &e0, &e1)) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
    else hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    return hipGetLastError();
}

// Launchers (defined in the .hip files).  All return hipError_t of the launch.
// Forward projection of the subset starting at slot `slot0` holding `nview`
// views.  mode 0: out = w .* (A x - y) (y, w may be null);
// mode 1: accumulate 1/2 sum w (A x - y)^2 into partials[part_off + block].
// ray_scaled (3D, mode 0): each ray's entry is further multiplied by the
// ray's scale (in-plane length factor times the row's cone factor), which a
// back-projection with BpEpi::ray_scaled then leaves out.
// With a batch, image b's y and w start at y + b yw_stride, its output at
// out + b out_stride and its partials at partials + b n_partials + part_off.
hipError_t launch_fp(const lalm_plan *p, int64_t slot0, int nview, const float *y,
                     const float *w, float *out, int mode, int64_t part_off,
                     int64_t *n_blocks_out, int check_status, hipStream_t st, int ray_scaled,
                     int64_t yw_stride, int64_t out_stride);

// The current scalar records (one per image) and the other set.
inline lalm::DevScalars *cur_sc(const lalm_plan *p) { return p->d_sc + (size_t)p->sc_cur * p->B; }
inline lalm::DevScalars *nxt_sc(const lalm_plan *p) { return p->d_sc + (size_t)(p->sc_cur ^ 1) * p->B; }
inline BatchStr batch_str(const lalm_plan *p) { return BatchStr{p->nvox, p->layT, p->layN, p->n_partials}; }
// The same forward projection, first taking the continuation decision of
// the previous step (every wave reduces the fused step kernel's partials in
// the same fixed order; one thread records it in the other scalar record)
// and reading the projector layouts of the candidate it selects.
hipError_t launch_fp_decide(const lalm_plan *p, int64_t slot0, int nview, const float *y, const float *w,
                            float *out, const ContArgs &cont, hipStream_t st, int64_t yw_stride,
                            int64_t out_stride);

// BP_LINES (2D): the partial back-projections of a STEP only; the fused
// step kernel (launch_step2d) follows.
enum BpMode { BP_PLAIN = 0, BP_INIT = 1, BP_STEP = 2, BP_LINES = 3 };
struct BpEpi {
    float scale;           // PLAIN: scale; INIT/STEP: M
    int accumulate;        // PLAIN
    float *out;            // PLAIN: output image
    float *G, *g;          // INIT/STEP
    const float *x;        // INIT/STEP: image for grad R
    float beta, inv_delta2;   // regularizer: beta, 1/delta^2
    ContArgs cont;
    int ray_scaled;        // 3D: r already carries each ray's scale (launch_fp ray_scaled)
    long long r_stride;    // batch: image b's residual starts at r + b r_stride
};
// BP_INIT includes its finite check (the scalars advance); BP_STEP leaves
// the continuation decision of the step to the next x-update or to
// launch_finalize.
hipError_t launch_bp(const lalm_plan *p, int64_t slot0, int nview, const float *r, int mode,
                     const BpEpi &e, hipStream_t st);
// Standalone continuation decision after the last BP_STEP of a call.
hipError_t launch_finalize(const lalm_plan *p, const ContArgs &c, hipStream_t st);
// 2D only: the two partial back-projections of a step, pointwise, fused
// with the next step's x-update.  x of this step is xs[sel] of the current
// scalar record (xs0 == xs1 when it is not a candidate); xw, when set,
// receives a copy of it.  G+, the g-update and the restart-indicator
// partials as BP_STEP; then, unless last, the next x for both values rho
// can take after the pending decision (restart: rho_0 = 1; continue:
// rho_{l+1}; one value with a fixed rho) into xo0 / xo1 and the two layout
// sets.  last: instead grad R(x) into the plan's gradient image.
hipError_t launch_step2d(const lalm_plan *p, const float *xs0, const float *xs1, float *xw, float *xo0,
                         float *xo1, const BpEpi &e, const float *denom, int nonneg, bool last,
                         hipStream_t st);

enum UpdMode { UPD_LAYOUT = 0, UPD_ONES = 1, UPD_STEP = 2 };
// UPD_STEP with cont != null first makes the pending continuation decision
// of the previous step (fused, every block computes it; one records it).
// vout != null: first of several inner FISTA iterations -- the step's
// result goes to vout and zout (the next momentum point) instead of x and
// the projector layouts.
hipError_t launch_update(const lalm_plan *p, int mode, float *x, const float *G, const float *g,
                         const float *denom, float beta, int nonneg, const ContArgs *cont,
                         hipStream_t st, float *vout = nullptr, float *zout = nullptr);
// Inner FISTA iteration i >= 2 on the constrained-denoising problem of the
// current step: v = P(z - (rho D_L (z - x) + s + grad R(z)) / (rho D_L + D_R)),
// s = rho G + (1 - rho) g; then zout = v + mom (v - v_prev) with v kept in
// v (in place), or, last, x = v and the projector layouts.
hipError_t launch_inner(const lalm_plan *p, const float *z, float *v, float *zout, float *x, const float *G,
                        const float *g, const float *denom, float beta, float inv_delta2, float mom, int nonneg,
                        bool last, hipStream_t st);
hipError_t launch_reg_grad(const lalm_plan *p, const float *x, float beta, float inv_delta2,
                           hipStream_t st);
hipError_t launch_set_scalars(const lalm_plan *p, int b, long long l, double rho, long long step, double alpha,
                              hipStream_t st);
// Barzilai-Borwein step at an iteration start: with compute, alpha in the
// current scalar record from s = x - x_prev, y = grad - grad_prev (FP64,
// fixed order); then x_prev, grad_prev <- x, grad.
hipError_t launch_bb(const lalm_plan *p, const float *x, const float *grad, float *x_prev, float *grad_prev,
                     const float *denom, bool compute, double alpha_min, hipStream_t st);

// FBP of a full-turn 2D fan-beam sinogram (subset-major y) into x.
hipError_t launch_fbp(const lalm_plan *p, const float *y, float *x, hipStream_t st);
int fbp_max_bins();

// FP64 reductions
hipError_t launch_sum_partials(const double *part, int64_t n, double *out, double scale,
                               hipStream_t st);
hipError_t launch_dot(const lalm_plan *p, const float *a, const float *b, int64_t n,
                      double *out, hipStream_t st);
hipError_t launch_reg_value(const lalm_plan *p, const float *x, double beta, double delta,
                            double *out, hipStream_t st);
hipError_t launch_rmsd(const lalm_plan *p, const float *a, const float *b, double radius,
                       double *out, hipStream_t st);
hipError_t launch_combine_cost(double *out3, const double *data, const double *reg,
                               hipStream_t st);

}  // namespace lalm
