// Learned warm start: a 3-level 2D U-Net on gfx950 with BF16 MFMA
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Every convolution-like product is one implicit GEMM kernel, C = A B, with
// operand gathers chosen by template parameters:
//   forward 3x3 conv    A(m = pixel, k = tap*Cin + c) = X[pixel + tap][c]
//                       B(k, n = cout)                = W[cout][tap][c]
//   input gradient      A(m = pixel, k = tap*Cout + o) = dZ[pixel - tap][o]
//                       B(k, n = cin)                 = W[o][tap][cin] (pre-transposed)
//   weight gradient     A(m = cout, k = pixel)        = dZ[pixel][cout]
//                       B(k, n = tap*Cin + c)         = X[pixel + tap][c]
//   transposed conv     the same with taps replaced by the 2x2 output phase.
// Tiles of BM x 32 (A) and BN x 32 (B) bf16 values are staged in LDS (double
// buffered), four waves each own a 32x32 block of C.  Concatenated inputs are
// read by channel range from two tensors (no copy).  Epilogues: bias + ReLU +
// bfloat16 store (forward), FP32 store split by channel range (input
// gradient), FP32 partial sums per K-split (weight gradient, reduced after in
// a fixed order: deterministic).  Activations and gradients are NHWC bf16.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "lalm_internal.h"
#include "lalm_unet.h"

namespace unet {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

constexpr int BK = 32;
constexpr int LDK = BK + 8;      // LDS row stride (bf16): 80-byte rows spread the banks

enum { A_CONV = 0, A_UPG = 1, A_MC = 2 };
enum { B_W = 0, B_NC = 1 };
enum { E_FWD = 0, E_DG = 1, E_WG = 2 };

struct GemmArgs {
    int M, N, K;
    // A operand sources (concatenated by channel: a1 has ac1, a2 has ac2)
    const bf16 *a1, *a2;
    int ac1, ac2;
    int gB, gH, gW;        // pixel grid of the A rows (A_CONV, A_UPG) or of K (A_MC, B_NC)
    int ntap, tsign;       // A_CONV: 9 or 1 taps, +1 forward / -1 flipped
    int ab;                // A_MC: >= 0 reads the gradient at the 2x2 output phase ab of a 2x grid
    // B operand
    const bf16 *w;         // B_W: [N][K]
    const bf16 *b1, *b2;   // B_NC sources (concatenated)
    int bc1, bc2, bntap;
    // epilogues
    const float *bias;
    int relu;
    bf16 *y;               // E_FWD output (channels N)
    bf16 *pool;            // conv3x3_kernel E_FWD: also the 2x2 max pooling of y (nullptr: none)
    int yup;               // E_FWD: 1 = store at output phase ab of a 2x grid; 2 = all four
                           // phases in one GEMM, column n = phase * yc + channel
    int yc;                // E_FWD, yup = 2: output channels (and bias entries)
    float *o1, *o2;        // E_DG: n < oc1 -> o1 (ld oc1), else o2 (ld N - oc1)
    int oc1;
    float *part;           // E_WG partials [split][M][N]
    int klen;              // E_WG: K per split (multiple of BK)
};

__device__ inline void pix_decode(int p, int H, int W, int &b, int &y, int &x)
{
    const int hw = H * W;
    b = p / hw;
    const int r = p - b * hw;
    y = r / W;
    x = r - y * W;
}

__device__ inline bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (bf16)0.0f;
    return z;
}

__device__ inline bf16x8 ld8(const bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// 8 consecutive channels c..c+7 of pixel (b, y, x) of a concatenated pair.
__device__ inline bf16x8 gather_ch(const bf16 *s1, const bf16 *s2, int c1, int c2, int H, int W, int b, int y,
                                   int x, int c)
{
    if (y < 0 || y >= H || x < 0 || x >= W) return zero8();
    const long long pix = ((long long)b * H + y) * W + x;
    if (c < c1) return ld8(s1 + pix * c1 + c);
    return ld8(s2 + pix * c2 + (c - c1));
}

// Per-slot state of an A-tile row that stays fixed over the K loop (A_CONV,
// A_UPG): whether the row exists, its pixel coordinates and the index of
// its pixel (A_UPG: of the pixel's top-left child on the 2x grid).
struct ARow {
    int ok, y, x, pix;
};

template <int AMODE, int BM>
__device__ inline void init_rows(const GemmArgs &g, int m0, int tid, ARow *rs)
{
    constexpr int NVT = BM * BK / 8;
    constexpr int NV = (NVT + 255) / 256;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int s = tid + v * 256;
        const int m = m0 + s / (BK / 8);
        ARow r{0, 0, 0, 0};
        if ((NVT % 256 == 0 || s < NVT) && m < g.M) {
            int b, y, x;
            pix_decode(m, g.gH, g.gW, b, y, x);
            r.ok = 1;
            r.y = y;
            r.x = x;
            r.pix = AMODE == A_UPG ? ((b * 2 * g.gH + 2 * y) * (2 * g.gW) + 2 * x) : m;
        }
        rs[v] = r;
    }
}

// A tile (BM rows x BK) -> registers, one bf16x8 per slot.  A_CONV / A_UPG:
// the K step's tap (or 2x2 phase) and channel range are uniform; a row's
// gather is one bounds test and one address per vector.  Every slot issues
// its load (an invalid one reads the start of its source), and the returned
// mask (bit v: slot v is valid) zeroes the invalid ones when they are stored
// to LDS: with neither a branch around a load nor a select on its value, a
// wave waits for a load only where its data is stored, and the compiler can
// count the loads in flight across loop iterations.
template <int AMODE, int BM>
__device__ inline unsigned load_a(const GemmArgs &g, const ARow *rs, int m0, int k0, int tid, bf16x8 *ra)
{
    constexpr int NVT = BM * BK / 8;                // vectors in the tile
    constexpr int NV = (NVT + 255) / 256;           // vectors per thread
    unsigned mask = 0;
    if (AMODE == A_MC) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int s = tid + v * 256;
            // slot -> (pixel kk, channel vector) ; channels along M
            const int kk = s / (BM / 8), mv = (s % (BM / 8)) * 8;
            const int k = k0 + kk, m = m0 + mv;
            const bool ok = (NVT % 256 == 0 || s < NVT) && k < g.K && m < g.M;
            long long off = 0;
            if (ok) {
                if (g.ab >= 0) {
                    int b, y, x;
                    pix_decode(k, g.gH, g.gW, b, y, x);
                    const long long pix = ((long long)b * 2 * g.gH + 2 * y + (g.ab >> 1)) * (2 * g.gW) + 2 * x + (g.ab & 1);
                    off = pix * g.ac1 + m;
                } else {
                    off = (long long)k * g.ac1 + m;
                }
            }
            ra[v] = ld8(g.a1 + off);
            mask |= ok ? 1u << v : 0u;
        }
        return mask;
    }
    // uniform over the block: source, channel offset and pixel shift of this K step
    const bf16 *src;
    int cs, c0, dy = 0, dx = 0, dpix;
    if (AMODE == A_CONV) {
        const int cin = g.ac1 + g.ac2;
        const int tap = k0 / cin, c = k0 - tap * cin;
        if (g.ntap == 9) {
            dy = g.tsign * (tap / 3 - 1);
            dx = g.tsign * (tap % 3 - 1);
        }
        const bool first = c < g.ac1;              // BK divides both channel counts
        src = first ? g.a1 : g.a2;
        cs = first ? g.ac1 : g.ac2;
        c0 = first ? c : c - g.ac1;
        dpix = dy * g.gW + dx;
    } else {                                        // A_UPG: k = ab * C + c over the 2x grid
        const int ab = k0 / g.ac1;
        src = g.a1;
        cs = g.ac1;
        c0 = k0 - ab * g.ac1;
        dpix = (ab >> 1) * 2 * g.gW + (ab & 1);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int s = tid + v * 256;
        const int q = (s % (BK / 8)) * 8;
        const ARow r = rs[v];
        bool ok = r.ok != 0;
        if (AMODE == A_CONV) {
            const int yy = r.y + dy, xx = r.x + dx;
            ok = ok && (unsigned)yy < (unsigned)g.gH && (unsigned)xx < (unsigned)g.gW;
        }
        const long long off = ok ? (long long)(r.pix + dpix) * cs + c0 + q : 0;
        ra[v] = ld8(src + off);
        mask |= ok ? 1u << v : 0u;
    }
    return mask;
}

template <int AMODE, int BM>
__device__ inline void store_a(bf16 *As, int tid, const bf16x8 *ra, unsigned mask)
{
    constexpr int NVT = BM * BK / 8;
    constexpr int NV = (NVT + 255) / 256;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int s = tid + v * 256;
        if (NVT % 256 != 0 && s >= NVT) continue;
        const bf16x8 val = (mask >> v) & 1u ? ra[v] : zero8();
        if (AMODE == A_MC) {
            const int kk = s / (BM / 8), mv = (s % (BM / 8)) * 8;
#pragma unroll
            for (int i = 0; i < 8; ++i) As[(mv + i) * LDK + kk] = val[i];
        } else {
            const int mm = s / (BK / 8), q = (s % (BK / 8)) * 8;
            *reinterpret_cast<bf16x8 *>(As + mm * LDK + q) = val;
        }
    }
}

// B tile (BN x BK) -> registers; BN * BK / 8 vectors spread over the
// threads.  B_W: every slot loads (an invalid one reads row 0) and the mask
// zeroes it at the store, as for A; B_NC: gathers under the lane mask.
template <int BMODE, int BN>
__device__ inline unsigned load_b(const GemmArgs &g, int n0, int k0, int tid, bf16x8 *rb)
{
    constexpr int NVT = BN * BK / 8;                // total vectors
    constexpr int NV = (NVT + 255) / 256;
    unsigned mask = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int s = tid + v * 256;
        if (BMODE == B_W) {
            const int nn = s / (BK / 8), q = (s % (BK / 8)) * 8;
            const int n = n0 + nn;
            const bool ok = (NVT % 256 == 0 || s < NVT) && n < g.N;
            rb[v] = ld8(g.w + (ok ? (long long)n * g.K + k0 + q : 0));
            mask |= ok ? 1u << v : 0u;
        } else {
            bf16x8 r = zero8();
            if (s < NVT) {
                const int kk = s / (BN / 8), nv = (s % (BN / 8)) * 8;
                const int k = k0 + kk, n = n0 + nv;
                if (k < g.K && n < g.N) {
                    int b, y, x;
                    pix_decode(k, g.gH, g.gW, b, y, x);
                    const int cin = g.bc1 + g.bc2;
                    const int tap = n / cin, c = n - tap * cin;
                    if (g.bntap == 9) {
                        y += tap / 3 - 1;
                        x += tap % 3 - 1;
                    }
                    r = gather_ch(g.b1, g.b2, g.bc1, g.bc2, g.gH, g.gW, b, y, x, c);
                }
            }
            rb[v] = r;
            mask |= 1u << v;
        }
    }
    return mask;
}

template <int BMODE, int BN>
__device__ inline void store_b(bf16 *Bs, int tid, const bf16x8 *rb, unsigned mask)
{
    constexpr int NVT = BN * BK / 8;
    constexpr int NV = (NVT + 255) / 256;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int s = tid + v * 256;
        if (s >= NVT) continue;
        const bf16x8 val = (mask >> v) & 1u ? rb[v] : zero8();
        if (BMODE == B_W) {
            const int nn = s / (BK / 8), q = (s % (BK / 8)) * 8;
            *reinterpret_cast<bf16x8 *>(Bs + nn * LDK + q) = val;
        } else {
            const int kk = s / (BN / 8), nv = (s % (BN / 8)) * 8;
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[(nv + i) * LDK + kk] = val[i];
        }
    }
}

// Four waves; each owns WMT x WNT accumulators of 32 x 32 (a 32 WMT x 32 WNT
// block of C), so one LDS stage feeds 2 WMT WNT independent MFMAs per wave.
template <int AMODE, int BMODE, int EPI, int BM, int BN, int WMT, int WNT>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    constexpr int NWM = BM / (32 * WMT), NWN = BN / (32 * WNT);
    static_assert(NWM * NWN == 4, "four waves");
    static_assert(BM * (BN + 8) <= 2 * (BM + BN) * LDK, "epilogue staging fits in the operand buffers");
    __shared__ __attribute__((aligned(16))) bf16 smem[2 * (BM + BN) * LDK];
    // A stages at smem + buf BM LDK, B stages after both A stages
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv % NWM, wn = wv / NWM;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    int kbeg = 0, kend = g.K;
    if (EPI == E_WG) {
        kbeg = blockIdx.z * g.klen;
        kend = min(g.K, kbeg + g.klen);
    }
    constexpr int NVA = (BM * BK / 8 + 255) / 256;
    constexpr int NVB = (BN * BK / 8 + 255) / 256;
    bf16x8 ra[NVA], rb[NVB];
    ARow rs[NVA];
    if (AMODE != A_MC) init_rows<AMODE, BM>(g, m0, tid, rs);
    floatx16 acc[WMT][WNT];
#pragma unroll
    for (int a = 0; a < WMT; ++a)
#pragma unroll
        for (int b = 0; b < WNT; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

    // two register stages take turns: the tile of step k + 2 is loaded while
    // step k computes, so two K tiles are in flight per block.  Steps run in
    // pairs; past the last K tile a step loads the last tile again, and a
    // step past kend (an odd step count) stores zeros, so the loop has no
    // branch around a load and one exit.
    bf16x8 ra2[NVA], rb2[NVB];
    unsigned ma = 0, mb = 0, ma2 = 0, mb2 = 0;
    const int klast = kbeg < kend ? kbeg + (kend - kbeg - 1) / BK * BK : kbeg;
    int buf = 0;
    if (kbeg < kend) {
        ma = load_a<AMODE, BM>(g, rs, m0, kbeg, tid, ra);
        mb = load_b<BMODE, BN>(g, n0, kbeg, tid, rb);
        ma2 = load_a<AMODE, BM>(g, rs, m0, min(kbeg + BK, klast), tid, ra2);
        mb2 = load_b<BMODE, BN>(g, n0, min(kbeg + BK, klast), tid, rb2);
    }
    auto step = [&](int k0, bf16x8 *xa, bf16x8 *xb, unsigned &mxa, unsigned &mxb) {
        const unsigned live = k0 < kend ? ~0u : 0u;
        bf16 *as_buf = smem + buf * (BM * LDK), *bs_buf = smem + 2 * BM * LDK + buf * (BN * LDK);
        store_a<AMODE, BM>(as_buf, tid, xa, mxa & live);
        store_b<BMODE, BN>(bs_buf, tid, xb, mxb & live);
        __syncthreads();
        const int kn = min(k0 + 2 * BK, klast);    // prefetch two tiles ahead
        mxa = load_a<AMODE, BM>(g, rs, m0, kn, tid, xa);
        mxb = load_b<BMODE, BN>(g, n0, kn, tid, xb);
        const bf16 *as = as_buf + (wm * 32 * WMT + (lane & 31)) * LDK + 8 * (lane >> 5);
        const bf16 *bs = bs_buf + (wn * 32 * WNT + (lane & 31)) * LDK + 8 * (lane >> 5);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8 a[WMT], b[WNT];
#pragma unroll
            for (int i = 0; i < WMT; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(as + i * 32 * LDK + kk);
#pragma unroll
            for (int j = 0; j < WNT; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(bs + j * 32 * LDK + kk);
#pragma unroll
            for (int i = 0; i < WMT; ++i)
#pragma unroll
                for (int j = 0; j < WNT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        buf ^= 1;
    };
    for (int k0 = kbeg; k0 < kend; k0 += 2 * BK) {
        step(k0, ra, rb, ma, mb);
        step(k0 + BK, ra2, rb2, ma2, mb2);
    }

    // element t of acc[i][j]: row wm*32*WMT + 32 i + 8(t/4) + 4(lane/32) + t%4,
    // column wn*32*WNT + 32 j + lane%32
    if (EPI == E_FWD) {
        __syncthreads();
        bf16 *Cs = smem;                           // BM x (BN + 8) bf16 staging
        constexpr int LDC = BN + 8;
#pragma unroll
        for (int j = 0; j < WNT; ++j) {
            const int cl = wn * 32 * WNT + 32 * j + (lane & 31), col = n0 + cl;
            const float bv = (col < g.N && g.bias) ? g.bias[g.yup == 2 ? col % g.yc : col] : 0.0f;
#pragma unroll
            for (int i = 0; i < WMT; ++i)
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int r = wm * 32 * WMT + 32 * i + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
                    float v = acc[i][j][t] + bv;
                    if (g.relu) v = fmaxf(v, 0.0f);
                    Cs[r * LDC + cl] = (bf16)v;
                }
        }
        __syncthreads();
        for (int s = tid; s < BM * (BN / 8); s += 256) {
            const int r = s / (BN / 8), cv = (s % (BN / 8)) * 8;
            const int m = m0 + r, n = n0 + cv;
            if (m >= g.M || n >= g.N) continue;
            long long pix = m;
            int ldy = g.N, c = n;
            if (g.yup) {
                int b, y, x, ab = g.ab;
                if (g.yup == 2) {                  // 8 columns never straddle a phase (yc % 8 == 0)
                    ab = n / g.yc;
                    c = n - ab * g.yc;
                    ldy = g.yc;
                }
                pix_decode(m, g.gH, g.gW, b, y, x);
                pix = ((long long)b * 2 * g.gH + 2 * y + (ab >> 1)) * (2 * g.gW) + 2 * x + (ab & 1);
            }
            *reinterpret_cast<bf16x8 *>(g.y + pix * ldy + c) = *reinterpret_cast<const bf16x8 *>(Cs + r * LDC + cv);
        }
    } else {
#pragma unroll
        for (int j = 0; j < WNT; ++j) {
            const int col = n0 + wn * 32 * WNT + 32 * j + (lane & 31);
            if (col >= g.N) continue;
            float *dst = EPI == E_WG ? g.part + (long long)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
            for (int i = 0; i < WMT; ++i)
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int m = m0 + wm * 32 * WMT + 32 * i + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
                    if (m >= g.M) continue;
                    if (EPI == E_DG) {
                        if (col < g.oc1) g.o1[(long long)m * g.oc1 + col] = acc[i][j][t];
                        else g.o2[(long long)m * (g.N - g.oc1) + (col - g.oc1)] = acc[i][j][t];
                    } else {
                        dst[(long long)m * g.N + col] = acc[i][j][t];
                    }
                }
        }
    }
}

// ------------------------------------------------------------------------
// 3x3 convolution (forward, or the input gradient with mirrored taps) as an
// implicit GEMM whose input tile is staged once per chunk of 32 channels.
// A block owns BN output channels and a run of consecutive TH x 16 pixel
// tiles.  The BN x 9 x cin weights (cin = 32 NCH) go to LDS once; the work
// is a sequence of items (tile, chunk of 32 input channels).  For each item
// the block stores the (TH + 2) x 18 pixel patch (zero outside the image),
// already in registers, to LDS and issues the loads of the item two places
// further on (two register sets take turns), so two patches are in flight
// while every wave runs 9 taps x 2 MFMA k-steps reading its operands from
// LDS: the nine taps re-read the patch in LDS instead of memory.  Same MFMA,
// operand layouts, summation order (chunk, tap, k-step) and epilogues as
// gemm_kernel (E_FWD: bias, ReLU, bf16 NHWC; E_DG: FP32 split output).
constexpr int CV_TW = 16;              // tile width (pixels)
constexpr int CV_LDP = 40;             // LDS stride per patch pixel / weight tap (bf16): 32 + 8
constexpr int CV_LDW = 9 * CV_LDP;     // LDS stride per weight row (9 taps)

template <int EPI, int BM, int BN, int NCH>
__global__ void __launch_bounds__(256) conv3x3_kernel(GemmArgs g, int tiles_per_block)
{
    static_assert((BM / 32) * (BN / 32) == 4, "four waves of 32x32");
    constexpr int TH = BM / CV_TW;                 // tile rows
    constexpr int PH = TH + 2, PW = CV_TW + 2;     // patch with a one-pixel halo
    constexpr int NPV = PH * PW * 4;               // patch vectors of 8 channels
    constexpr int NP = (NPV + 255) / 256;          // per thread
    constexpr int NWV = NCH * BN * 36;             // weight vectors
    constexpr int NW = (NWV + 255) / 256;
    constexpr int LDC = BN + 8;
    __shared__ __attribute__((aligned(16))) bf16 Ps[PH * PW * CV_LDP];
    __shared__ __attribute__((aligned(16))) bf16 Ws[NCH * BN * CV_LDW];
    __shared__ __attribute__((aligned(16))) bf16 Cs[EPI == E_FWD ? BM * LDC : 8];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv % (BM / 32), wn = wv / (BM / 32);
    const int ntx = (g.gW + CV_TW - 1) / CV_TW, nty = (g.gH + TH - 1) / TH;
    const int ntiles = g.gB * nty * ntx;
    const int t0 = blockIdx.x * tiles_per_block;
    const int nitem = (min(ntiles, t0 + tiles_per_block) - t0) * NCH;   // items (tile, chunk)
    if (nitem <= 0) return;
    const int n0 = blockIdx.y * BN;
    const int cin = g.ac1 + g.ac2;                 // 32 NCH

    // the patch of item it -> registers, one vector per slot
    auto load_patch = [&](int it, bf16x8 *rp) {
        const int tt = t0 + it / NCH, cc = it % NCH;
        const int tx0 = (tt % ntx) * CV_TW;
        const int rest = tt / ntx;
        const int ty0 = (rest % nty) * TH, b = rest / nty;
        const bool first = 32 * cc < g.ac1;        // 32 divides both channel counts
        const bf16 *src = first ? g.a1 : g.a2;
        const int cs = first ? g.ac1 : g.ac2, c0 = first ? 32 * cc : 32 * cc - g.ac1;
#pragma unroll
        for (int v = 0; v < NP; ++v) {
            const int sl = tid + v * 256;
            const int q = sl & 3, pp = sl >> 2;
            const int yy = ty0 + pp / PW - 1, xx = tx0 + pp % PW - 1;
            bf16x8 val = zero8();
            if ((NPV % 256 == 0 || sl < NPV) && (unsigned)yy < (unsigned)g.gH && (unsigned)xx < (unsigned)g.gW)
                val = ld8(src + (((long long)b * g.gH + yy) * g.gW + xx) * cs + c0 + 8 * q);
            rp[v] = val;
        }
    };

    bf16x8 ra[NP], rb[NP];
    load_patch(0, ra);
    if (nitem > 1) load_patch(1, rb);
    {
        // all weights, [chunk][N][tap][32 channels], rows from K = tap * cin + c
        bf16x8 rw[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const int sl = tid + v * 256;
            const int q = sl & 3, tp = (sl >> 2) % 9, row = sl / 36;   // row = chunk * BN + nn
            const int cc = row / BN, nn = row - cc * BN;
            bf16x8 val = zero8();
            if ((NWV % 256 == 0 || sl < NWV) && n0 + nn < g.N)
                val = ld8(g.w + (long long)(n0 + nn) * g.K + tp * cin + 32 * cc + 8 * q);
            rw[v] = val;
        }
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            const int sl = tid + v * 256;
            if (NWV % 256 != 0 && sl >= NWV) continue;
            const int q = sl & 3, tp = (sl >> 2) % 9, row = sl / 36;
            *reinterpret_cast<bf16x8 *>(Ws + row * CV_LDW + tp * CV_LDP + 8 * q) = rw[v];
        }
    }

    // this lane's A row: tile pixel wm*32 + lane%32 (row-major TH x 16)
    const int pr = wm * 32 + (lane & 31);
    const int py = pr / CV_TW, px = pr % CV_TW;
    const int col = n0 + wn * 32 + (lane & 31);
    float bv = 0.0f;
    if (EPI == E_FWD) bv = (col < g.N && g.bias) ? g.bias[col] : 0.0f;
    floatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;

    // one item: its patch rp -> LDS, loads of item it + 2 into rp, the MFMAs,
    // and after the tile's last chunk the epilogue
    auto item = [&](int it, bf16x8 *rp) {
        __syncthreads();                           // the previous item's readers are done
#pragma unroll
        for (int v = 0; v < NP; ++v) {
            const int sl = tid + v * 256;
            if (NPV % 256 != 0 && sl >= NPV) continue;
            *reinterpret_cast<bf16x8 *>(Ps + (sl >> 2) * CV_LDP + 8 * (sl & 3)) = rp[v];
        }
        __syncthreads();
        if (it + 2 < nitem) load_patch(it + 2, rp);  // in flight during two items
        const int c = it % NCH;
        const bf16 *ws = Ws + (c * BN + wn * 32 + (lane & 31)) * CV_LDW + 8 * (lane >> 5);
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            const int dy = g.tsign * (tp / 3 - 1), dx = g.tsign * (tp % 3 - 1);
            const bf16 *ps = Ps + ((py + 1 + dy) * PW + px + 1 + dx) * CV_LDP + 8 * (lane >> 5);
#pragma unroll
            for (int kk = 0; kk < 32; kk += 16) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(ps + kk);
                const bf16x8 bw = *reinterpret_cast<const bf16x8 *>(ws + tp * CV_LDP + kk);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bw, acc, 0, 0, 0);
            }
        }
        if (c != NCH - 1) return;
        // element q of acc: tile pixel wm*32 + 8(q/4) + 4(lane/32) + q%4, column col
        const int tt = t0 + it / NCH;
        const int tx0 = (tt % ntx) * CV_TW;
        const int rest = tt / ntx;
        const int ty0 = (rest % nty) * TH, b = rest / nty;
        if (EPI == E_FWD) {
            // Cs is rewritten only after the two barriers at the top of the
            // next item, so the reads below are done by then
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = wm * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                float v = acc[q] + bv;
                if (g.relu) v = fmaxf(v, 0.0f);
                Cs[r * LDC + wn * 32 + (lane & 31)] = (bf16)v;
            }
            __syncthreads();
            for (int sl = tid; sl < BM * (BN / 8); sl += 256) {
                const int r = sl / (BN / 8), cv = (sl % (BN / 8)) * 8;
                const int y = ty0 + r / CV_TW, x = tx0 + r % CV_TW, n = n0 + cv;
                if (y >= g.gH || x >= g.gW || n >= g.N) continue;
                const long long pix = ((long long)b * g.gH + y) * g.gW + x;
                *reinterpret_cast<bf16x8 *>(g.y + pix * g.N + n) = *reinterpret_cast<const bf16x8 *>(Cs + r * LDC + cv);
            }
            if (g.pool) {
                // 2x2 max pooling of the tile (its rows and columns start even;
                // H and W are even): the window in scan order, a later value
                // taken only when larger, as pool_fwd_kernel does
                const int Ho = g.gH / 2, Wo = g.gW / 2;
                for (int sl = tid; sl < (TH / 2) * (CV_TW / 2) * (BN / 8); sl += 256) {
                    const int cv = (sl % (BN / 8)) * 8, q = sl / (BN / 8);
                    const int qy = q / (CV_TW / 2), qx = q % (CV_TW / 2);
                    const int yo = ty0 / 2 + qy, xo = tx0 / 2 + qx, n = n0 + cv;
                    if (yo >= Ho || xo >= Wo || n >= g.N) continue;
                    const int r0 = 2 * qy * CV_TW + 2 * qx;
                    bf16x8 m = *reinterpret_cast<const bf16x8 *>(Cs + r0 * LDC + cv);
                    const int rr[3] = {r0 + 1, r0 + CV_TW, r0 + CV_TW + 1};
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const bf16x8 v = *reinterpret_cast<const bf16x8 *>(Cs + rr[k] * LDC + cv);
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if ((float)v[i] > (float)m[i]) m[i] = v[i];
                    }
                    const long long po = ((long long)b * Ho + yo) * Wo + xo;
                    *reinterpret_cast<bf16x8 *>(g.pool + po * g.N + n) = m;
                }
            }
        } else if (col < g.N) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = wm * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                const int y = ty0 + r / CV_TW, x = tx0 + r % CV_TW;
                if (y >= g.gH || x >= g.gW) continue;
                const long long m = ((long long)b * g.gH + y) * g.gW + x;
                if (col < g.oc1) g.o1[m * g.oc1 + col] = acc[q];
                else g.o2[m * (g.N - g.oc1) + (col - g.oc1)] = acc[q];
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    };

    for (int it = 0;; it += 2) {
        item(it, ra);
        if (it + 1 >= nitem) break;
        item(it + 1, rb);
        if (it + 2 >= nitem) break;
    }
}

template <int AMODE, int BMODE, int EPI>
hipError_t gemm(const GemmArgs &g, int nsplit, hipStream_t st)
{
    // wide tiles, four accumulators per wave, wherever N fills them
    if (g.N <= 32) {
        dim3 grd((g.M + 127) / 128, (g.N + 31) / 32, nsplit);
        hipLaunchKernelGGL((gemm_kernel<AMODE, BMODE, EPI, 128, 32, 1, 1>), grd, dim3(256), 0, st, g);
    } else if (g.N <= 64) {
        dim3 grd((g.M + 255) / 256, (g.N + 63) / 64, nsplit);
        hipLaunchKernelGGL((gemm_kernel<AMODE, BMODE, EPI, 256, 64, 2, 2>), grd, dim3(256), 0, st, g);
    } else {
        dim3 grd((g.M + 127) / 128, (g.N + 127) / 128, nsplit);
        hipLaunchKernelGGL((gemm_kernel<AMODE, BMODE, EPI, 128, 128, 2, 2>), grd, dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Weight gradient dW[m][n] = sum_k A[k][m] B[k][n] over pixels k (split K):
// A = the output gradient dz (channels m; A_MC, or its 2x2 phase ab of a 2x
// grid), B = the input at the tap of column n (B_NC).  Same MFMA layout as
// gemm_kernel.  Every thread keeps the pixel of each of its slots as
// (image row r = b*H + y, y, x) and steps it by BK pixels per K step, and
// the tap / channel / source of each B slot is fixed for the kernel, so the
// K loop does no integer division.  Two pixels per thread and slot are
// loaded, so the transposing LDS stores write packed pairs.
struct PixState {
    int r, y, x, k;
};

__device__ inline PixState pix_init(int k, int H, int W)
{
    PixState p;
    p.k = k;
    p.r = k / W;
    p.x = k - p.r * W;
    p.y = p.r % H;
    return p;
}

__device__ inline void pix_advance(PixState &p, int by, int H, int W)
{
    p.k += by;
    p.x += by;
    while (p.x >= W) {
        p.x -= W;
        ++p.r;
        if (++p.y == H) p.y = 0;
    }
}

template <int BM, int BN>
__global__ void __launch_bounds__(256) wgrad_kernel(GemmArgs g)
{
    static_assert((BM / 32) * (BN / 32) == 4, "four waves of 32x32");
    static_assert((LDK / 2) % 8 == 4 && BK == 32, "the bank rotation of store2 assumes 20-word rows and 16 pixel pairs");
    constexpr int PA = BM * BK / 16;                 // A pixel pairs x channel vectors in the tile
    constexpr int PB = BN * BK / 16;
    constexpr int NA = (PA + 255) / 256, NB = (PB + 255) / 256;
    __shared__ __attribute__((aligned(16))) bf16 As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) bf16 Bs[2][BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv % (BM / 32), wn = wv / (BM / 32);
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * g.klen, kend = min(g.K, kbeg + g.klen);
    const int H = g.gH, W = g.gW;

    // A slots: pixel pair kp (pixels 2kp, 2kp+1 of the tile), channels
    // mv..mv+7; the pair index runs fastest over the lanes (see store2)
    PixState pa[NA][2];
    int am[NA];
    bool aon[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) {
        const int s = tid + 256 * v;
        aon[v] = PA % 256 == 0 || s < PA;
        const int kp = s % (BK / 2);
        am[v] = m0 + (s / (BK / 2)) * 8;
        pa[v][0] = pix_init(kbeg + 2 * kp, H, W);
        pa[v][1] = pix_init(kbeg + 2 * kp + 1, H, W);
    }
    // B slots: the column block fixes the tap, channel and source
    PixState pb[NB][2];
    const bf16 *bsrc[NB];
    int bcs[NB], bcc[NB], bdy[NB], bdx[NB];
    bool bon[NB];
#pragma unroll
    for (int v = 0; v < NB; ++v) {
        const int s = tid + 256 * v;
        const int kp = s % (BK / 2), n = n0 + (s / (BK / 2)) * 8;
        bon[v] = (PB % 256 == 0 || s < PB) && n < g.N;
        const int cin = g.bc1 + g.bc2;
        const int tap = bon[v] ? n / cin : 0, c = bon[v] ? n - tap * cin : 0;
        bdy[v] = g.bntap == 9 ? tap / 3 - 1 : 0;
        bdx[v] = g.bntap == 9 ? tap % 3 - 1 : 0;
        const bool first = c < g.bc1;
        bsrc[v] = first ? g.b1 : g.b2;
        bcs[v] = first ? g.bc1 : g.bc2;
        bcc[v] = first ? c : c - g.bc1;
        pb[v][0] = pix_init(kbeg + 2 * kp, H, W);
        pb[v][1] = pix_init(kbeg + 2 * kp + 1, H, W);
    }

    auto load_a2 = [&](bf16x8 (*ra)[2]) {
#pragma unroll
        for (int v = 0; v < NA; ++v)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const PixState &p = pa[v][h];
                bf16x8 r = zero8();
                if (aon[v] && p.k < kend && am[v] < g.M) {
                    const long long pix = g.ab >= 0 ? (long long)(2 * p.r + (g.ab >> 1)) * (2 * W) + 2 * p.x + (g.ab & 1)
                                                    : (long long)p.k;
                    r = ld8(g.a1 + pix * g.ac1 + am[v]);
                }
                ra[v][h] = r;
            }
    };
    auto load_b2 = [&](bf16x8 (*rb)[2]) {
#pragma unroll
        for (int v = 0; v < NB; ++v)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const PixState &p = pb[v][h];
                const int yy = p.y + bdy[v], xx = p.x + bdx[v];
                bf16x8 r = zero8();
                if (bon[v] && p.k < kend && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W)
                    r = ld8(bsrc[v] + ((long long)(p.r + bdy[v]) * W + xx) * bcs[v] + bcc[v]);
                rb[v][h] = r;
            }
    };
    auto advance = [&]() {
#pragma unroll
        for (int v = 0; v < NA; ++v) {
            pix_advance(pa[v][0], BK, H, W);
            pix_advance(pa[v][1], BK, H, W);
        }
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            pix_advance(pb[v][0], BK, H, W);
            pix_advance(pb[v][1], BK, H, W);
        }
    };
    // transposed stores: element e of the two pixels' vectors -> one 32-bit
    // word of row mv + e.  The 16 lanes of a channel group write 16
    // consecutive words of one row; the next group's rows are 8 further on,
    // 160 words, the same banks, so odd groups write their elements rotated
    // by 4 (rows 4 or 12 apart, 16 banks further): a 32-lane half-wave
    // covers the 32 banks once.
    auto store2 = [&](bf16 *S, int n_pairs, int s, const bf16x8 &v0, const bf16x8 &v1) {
        if (s >= n_pairs) return;
        const int kp = s % (BK / 2), grp = s / (BK / 2), mv = grp * 8;
        const bool odd = grp & 1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
            const int e = odd ? (i + 4) & 7 : i;
            bf16x2 pr;
            pr[0] = odd ? v0[(i + 4) & 7] : v0[i];
            pr[1] = odd ? v1[(i + 4) & 7] : v1[i];
            *reinterpret_cast<bf16x2 *>(S + (mv + e) * LDK + 2 * kp) = pr;
        }
    };

    bf16x8 ra[NA][2], rb[NB][2];
    floatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    int buf = 0;
    if (kbeg < kend) {
        load_a2(ra);
        load_b2(rb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int v = 0; v < NA; ++v) store2(As[buf], PA, tid + 256 * v, ra[v][0], ra[v][1]);
#pragma unroll
        for (int v = 0; v < NB; ++v) store2(Bs[buf], PB, tid + 256 * v, rb[v][0], rb[v][1]);
        __syncthreads();
        if (k0 + BK < kend) {                      // prefetch the next tile
            advance();
            load_a2(ra);
            load_b2(rb);
        }
        const bf16 *as = As[buf] + (wm * 32 + (lane & 31)) * LDK + 8 * (lane >> 5);
        const bf16 *bs = Bs[buf] + (wn * 32 + (lane & 31)) * LDK + 8 * (lane >> 5);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(as + kk);
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(bs + kk);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        buf ^= 1;
    }
    const int col = n0 + wn * 32 + (lane & 31);
    if (col >= g.N) return;
    float *dst = g.part + (long long)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int m = m0 + wm * 32 + 8 * (t >> 2) + 4 * (lane >> 5) + (t & 3);
        if (m < g.M) dst[(long long)m * g.N + col] = acc[t];
    }
}

// 3x3 convolutions with 32 output channels and up to 64 input channels take
// the patch-staged kernel (its weights for 32 output channels fit beside
// the patch); wider outputs keep the generic implicit GEMM, whose smaller
// LDS footprint keeps more blocks resident (measured faster for 64 and 128
// channels).  Tiles per block: up to 4, as long as the grid keeps about
// 4096 blocks (16 per CU).
template <int EPI>
hipError_t conv3x3(const GemmArgs &g, hipStream_t st, bool fused_pool = false)
{
    const int cin = g.ac1 + g.ac2;
    if (g.N > 32 || (cin != 32 && cin != 64)) {
        if (fused_pool) return hipErrorInvalidValue;   // only the patch kernel pools
        return gemm<A_CONV, B_W, EPI>(g, 1, st);
    }
    const int ntiles = g.gB * ((g.gH + 7) / 8) * ((g.gW + CV_TW - 1) / CV_TW);
    const int tpb = std::max(1, std::min(4, ntiles / 4096));
    const dim3 grd((ntiles + tpb - 1) / tpb, 1);
    if (cin == 32) hipLaunchKernelGGL((conv3x3_kernel<EPI, 128, 32, 1>), grd, dim3(256), 0, st, g, tpb);
    else hipLaunchKernelGGL((conv3x3_kernel<EPI, 128, 32, 2>), grd, dim3(256), 0, st, g, tpb);
    return hipGetLastError();
}

// ------------------------------------------------------------ VALU kernels

// first layer: 3x3 conv 1 -> 32 with ReLU, x FP32 [P] (images), out bf16
// [P][32].  On the matrix cores: 32 consecutive pixels x 32 output channels
// are one 32x32x16 MFMA, K = the 9 taps (zero-padded to 16): lanes 0-31 give
// taps 0-7 of their pixel, lanes 32-63 tap 8 and zeros; the B operand
// (bfloat16 weights, channel lane % 32) is loaded once.  A wave takes
// C1_G groups of 32 pixels and issues all their input loads first.  Inputs
// in_scale * x and weights rounded to bfloat16, FP32 accumulation.  Each
// 32 x 32 result goes through LDS so every pixel's 64 bytes are written by
// two lanes together.
constexpr int C1_G = 4;

__global__ void __launch_bounds__(256) conv1_mfma_kernel(const float *x, float in_scale, const float *w,
                                                         const float *bias, bf16 *out, int B, int H, int W)
{
    __shared__ __attribute__((aligned(16))) bf16 Cs[4][32 * 40];   // per wave: 32 pixels x 32 channels (+8)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long P = (long long)B * H * W;
    const int c = lane & 31, kh = lane >> 5;
    bf16x8 bw;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int t = 8 * kh + j;
        bw[j] = (bf16)(t < 9 ? w[c * 9 + t] : 0.0f);
    }
    const float bv = bias[c];
    const long long base = ((long long)blockIdx.x * 4 + wv) * (32 * C1_G);   // first pixel of this wave
    if (base >= P) return;                                                  // whole waves only
    bf16x8 a[C1_G];
#pragma unroll
    for (int gi = 0; gi < C1_G; ++gi) {
        const long long p = base + 32 * gi + c;
        a[gi] = zero8();
        if (p < P) {
            int b, y, xx;
            pix_decode((int)p, H, W, b, y, xx);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int t = 8 * kh + j;
                if (t < 9) {
                    const int yy = y + t / 3 - 1, xq = xx + t % 3 - 1;
                    float v = 0.0f;
                    if (yy >= 0 && yy < H && xq >= 0 && xq < W) v = in_scale * x[((long long)b * H + yy) * W + xq];
                    a[gi][j] = (bf16)v;
                }
            }
        }
    }
    bf16 *cs = Cs[wv];
#pragma unroll
    for (int gi = 0; gi < C1_G; ++gi) {
        floatx16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[gi], bw, acc, 0, 0, 0);
        // element q: pixel 8(q/4) + 4(lane/32) + q%4 of the group, channel lane % 32
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = 8 * (q >> 2) + 4 * kh + (q & 3);
            cs[r * 40 + c] = (bf16)fmaxf(acc[q] + bv, 0.0f);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        // 32 pixels x 64 bytes: lane takes pixel lane/2, half lane%2 (two 16-byte chunks)
        const int r = lane >> 1, h = lane & 1;
        const long long p = base + 32 * gi + r;
        if (p < P) {
            bf16 *dst = out + p * 32 + 16 * h;
            *reinterpret_cast<bf16x8 *>(dst) = *reinterpret_cast<const bf16x8 *>(cs + r * 40 + 16 * h);
            *reinterpret_cast<bf16x8 *>(dst + 8) = *reinterpret_cast<const bf16x8 *>(cs + r * 40 + 16 * h + 8);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");   // reads done before the next group's writes
    }
}

// gradient of the first layer's weights and biases over a chunk of pixels:
// part[blk][c*10 + t] = sum_p dz[p][c] * u[p + tap t] (t < 9), bias at t = 9,
// with u the scaled, bfloat16-rounded input.  256 threads: 4 vectors of 8
// channels x 64 pixel lanes; the lanes are combined in fixed order.
__global__ void __launch_bounds__(256) conv1_wgrad_kernel(const float *x, float in_scale, const bf16 *dz,
                                                          float *part, int B, int H, int W, int chunk)
{
    __shared__ float red[64 * 32];
    const int cv = threadIdx.x & 3, pl = threadIdx.x >> 2;
    const long long P = (long long)B * H * W;
    const long long p0 = (long long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    float acc[8][10];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int t = 0; t < 10; ++t) acc[i][t] = 0.0f;
    for (long long p = p0 + pl; p < p1; p += 64) {
        int b, y, xx;
        pix_decode((int)p, H, W, b, y, xx);
        float u[10];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xq = xx + t % 3 - 1;
            u[t] = (yy >= 0 && yy < H && xq >= 0 && xq < W)
                       ? (float)(bf16)(in_scale * x[((long long)b * H + yy) * W + xq]) : 0.0f;
        }
        u[9] = 1.0f;
        const bf16x8 d = ld8(dz + p * 32 + cv * 8);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float di = (float)d[i];
#pragma unroll
            for (int t = 0; t < 10; ++t) acc[i][t] = fmaf(di, u[t], acc[i][t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 10; ++t) {
#pragma unroll
        for (int i = 0; i < 8; ++i) red[pl * 32 + cv * 8 + i] = acc[i][t];
        __syncthreads();
        if (threadIdx.x < 32) {
            float s = 0.0f;
            for (int k = 0; k < 64; ++k) s += red[k * 32 + threadIdx.x];
            part[(long long)blockIdx.x * 320 + threadIdx.x * 10 + t] = s;
        }
        __syncthreads();
    }
}

// 2x2 max pooling, NHWC bf16; one thread per output pixel and 8 channels
__global__ void pool_fwd_kernel(const bf16 *in, bf16 *out, int B, int H, int W, int C)
{
    const int Ho = H / 2, Wo = W / 2, CV = C / 8;
    const long long n = (long long)B * Ho * Wo * CV;
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int cv = (int)(s % CV) * 8;
    const long long po = s / CV;
    int b, y, x;
    pix_decode((int)po, Ho, Wo, b, y, x);
    const long long base = ((long long)b * H + 2 * y) * W + 2 * x;
    bf16x8 m = ld8(in + base * C + cv);
    const long long q[3] = {base + 1, base + W, base + W + 1};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bf16x8 v = ld8(in + q[k] * C + cv);
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if ((float)v[i] > (float)m[i]) m[i] = v[i];
    }
    *reinterpret_cast<bf16x8 *>(out + po * C + cv) = m;
}

// pooling backward: g (FP32, pooled grid) goes to the first maximum of its
// window in scan order, added into acc (FP32, full grid)
__global__ void pool_bwd_kernel(const bf16 *in, const float *g, float *acc, int B, int H, int W, int C)
{
    const int Ho = H / 2, Wo = W / 2;
    const long long n = (long long)B * Ho * Wo * C;
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int c = (int)(s % C);
    const long long po = s / C;
    int b, y, x;
    pix_decode((int)po, Ho, Wo, b, y, x);
    const long long base = ((long long)b * H + 2 * y) * W + 2 * x;
    const long long q[4] = {base, base + 1, base + W, base + W + 1};
    int best = 0;
    float mv = (float)in[q[0] * C + c];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        const float v = (float)in[q[k] * C + c];
        if (v > mv) { mv = v; best = k; }
    }
    acc[q[best] * C + c] += g[s];
}

// dz = bf16(g) where act > 0 (or everywhere when act is null)
// dz = bf16(g) where the ReLU was active (act > 0; every element when act
// is null); 8 elements per thread
__global__ void mask_to_bf16_kernel(const float *g, const bf16 *act, bf16 *dz, long long n8)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const float4 lo = reinterpret_cast<const float4 *>(g)[2 * i];
    const float4 hi = reinterpret_cast<const float4 *>(g)[2 * i + 1];
    const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    bf16x8 o;
    if (act) {
        const bf16x8 a = ld8(act + 8 * i);
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = (bf16)((float)a[k] > 0.0f ? v[k] : 0.0f);
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = (bf16)v[k];
    }
    *reinterpret_cast<bf16x8 *>(dz + 8 * i) = o;
}

// stored bfloat16 tensor -> FP32 copy (exact)
__global__ void bf16_to_f32_kernel(const bf16 *src, float *dst, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// head: out = x + sum_c a[p][c] w[c] + b; with a target also the loss
// partials and dout = 2 s^2 (out - t) mask / n
__global__ void head_kernel(const float *x, float inv_scale, int nonneg, const bf16 *a, const float *w,
                            const float *bias, float *out, const float *target, const uint8_t *mask,
                            double s2_over_n, float *dout, double *lpart, long long P, int HW)
{
    __shared__ double red[256];
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (p < P) {
        float acc = bias[0];
        const bf16 *ap = a + p * 32;
#pragma unroll
        for (int c = 0; c < 32; ++c) acc = fmaf((float)ap[c], (float)(bf16)w[c], acc);
        const float o = fmaf(acc, inv_scale, x[p]);
        if (out) out[p] = nonneg ? fmaxf(o, 0.0f) : o;
        if (target) {
            const float mk = mask[p % HW] ? 1.0f : 0.0f;
            const double e = ((double)o - (double)target[p]) * mk;
            l = e * e * s2_over_n;
            // gradient w.r.t. the head's output (scaled units)
            dout[p] = (float)(2.0 * s2_over_n * e * (double)inv_scale);
        }
    }
    if (!target) return;
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// head backward: dz_d1b[p][c] = dout[p] w[c] masked by a > 0
__global__ void head_bwd_kernel(const float *dout, const bf16 *a, const float *w, bf16 *dz, long long P)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P * 32) return;
    const long long p = s / 32;
    const int c = (int)(s % 32);
    const float v = ((float)a[s] > 0.0f) ? dout[p] * (float)(bf16)w[c] : 0.0f;
    dz[s] = (bf16)v;
}

// column sums over a chunk of pixels: part[blk][c] = sum_p v[p][c], or
// sum_p mul[p] v[p][c] when mul is given (v: [P][C] bf16).  256 threads: C/8
// channel vectors x 2048/C pixel lanes, lanes combined in fixed order.
template <int C>
__global__ void __launch_bounds__(256) colsum_kernel(const bf16 *v, const float *mul, long long P, int chunk,
                                                     float *part)
{
    constexpr int CV = C / 8, PL = 256 / CV;
    __shared__ float red[PL * C];
    const int cv = threadIdx.x % CV, pl = threadIdx.x / CV;
    const long long p0 = (long long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
    for (long long p = p0 + pl; p < p1; p += PL) {
        const bf16x8 x = ld8(v + p * C + cv * 8);
        const float m = mul ? mul[p] : 1.0f;
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = fmaf(m, (float)x[i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) red[pl * C + cv * 8 + i] = acc[i];
    __syncthreads();
    if (threadIdx.x < C) {
        float s = 0.0f;
        for (int k = 0; k < PL; ++k) s += red[k * C + threadIdx.x];
        part[(long long)blockIdx.x * C + threadIdx.x] = s;
    }
}

// part[blk] = sum of v over a chunk (fixed-order tree)
__global__ void __launch_bounds__(256) sum_chunk_kernel(const float *v, long long P, int chunk, float *part)
{
    __shared__ float red[256];
    const long long p0 = (long long)blockIdx.x * chunk, p1 = min(P, p0 + chunk);
    float s = 0.0f;
    for (long long p = p0 + threadIdx.x; p < p1; p += 256) s += v[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[i] = sum_s part[s][i] in a fixed order: 32 outputs x 8 split lanes per
// block (lane j sums splits j, j+8, ...), lanes combined in order
// out[i] = sum over the ns splits of part[k][i], in a fixed order: a block
// of 1024 threads takes 32 outputs; thread (k-lane sy, output ox) sums
// splits sy, sy + 32, ... into eight running sums (eight loads in flight),
// adds them pairwise, and the first wave adds the 32 k-lanes in order.
__global__ void __launch_bounds__(1024) reduce_parts_kernel(const float *part, int ns, long long n, float *out)
{
    __shared__ float red[32][33];
    const int ox = threadIdx.x & 31, sy = threadIdx.x >> 5;
    const long long i = (long long)blockIdx.x * 32 + ox;
    float s[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (i < n) {
        int k = sy;
        for (; k + 7 * 32 < ns; k += 8 * 32) {
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] += part[(long long)(k + 32 * u) * n + i];
        }
        for (; k < ns; k += 32) s[0] += part[(long long)k * n + i];
    }
    red[sy][ox] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (sy == 0 && i < n) {
        float t = red[0][ox];
#pragma unroll
        for (int j = 1; j < 32; ++j) t += red[j][ox];
        out[i] = t;
    }
}

__global__ void sum_double_kernel(const double *p, int n, double *out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// FP32 master weights -> bf16 forward copy and the pre-transposed
// input-gradient copies: 3x3 [cin][tap][cout] (the gather applies the
// negated tap offset), 2x2 [cin][phase][cout].  All layers in one launch:
// element i of the concatenated weight list belongs to the layer whose
// prefix range holds it.
constexpr int kPrepMax = 16;
struct PrepTable {
    int n;
    long long start[kPrepMax + 1];
    const float *src[kPrepMax];
    bf16 *wf[kPrepMax], *wd[kPrepMax];
    int cout[kPrepMax], cin[kPrepMax], up[kPrepMax];
};
__global__ void prep_all_kernel(PrepTable T)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T.start[T.n]) return;
    int L = 0;
    while (i >= T.start[L + 1]) ++L;
    const long long k = i - T.start[L];
    const int cout = T.cout[L], cin = T.cin[L];
    const int c = (int)(k % cin);
    const bf16 v = (bf16)T.src[L][k];
    T.wf[L][k] = v;
    if (T.up[L]) {
        const int o = (int)((k / cin) % cout);
        const int ab = (int)(k / ((long long)cout * cin));
        T.wd[L][((long long)c * 4 + ab) * cout + o] = v;     // [c][ab][o]
    } else {
        const int tap = (int)((k / cin) % 9);
        const int o = (int)(k / (9LL * cin));
        T.wd[L][((long long)c * 9 + tap) * cout + o] = v;    // [c][tap][o]
    }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, long long n, float lr, float bc1,
                            float bc2)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

// first layer gradient [c][t] (t < 9 weights, t = 9 bias) -> flat layout
__global__ void scatter_conv1_kernel(const float *src, float *gw, float *gb)
{
    const int o = threadIdx.x;
    if (o >= 320) return;
    const int c = o / 10, t = o % 10;
    if (t < 9) gw[c * 9 + t] = src[o];
    else gb[c] = src[o];
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace unet

// ------------------------------------------------------------------ network

using namespace unet;

namespace {

struct LayerDef { const char *name; int kind; int cin, cout; };   // kind 0 conv, 1 up, 2 head
const LayerDef kLayers[] = {
    {"e1a", 0, 1, 32}, {"e1b", 0, 32, 32}, {"e2a", 0, 32, 64}, {"e2b", 0, 64, 64},
    {"e3a", 0, 64, 128}, {"e3b", 0, 128, 128}, {"up2", 1, 128, 64}, {"d2a", 0, 128, 64},
    {"d2b", 0, 64, 64}, {"up1", 1, 64, 32}, {"d1a", 0, 64, 32}, {"d1b", 0, 32, 32}, {"head", 2, 32, 1}};
constexpr int kNL = 13;
enum { E1A, E1B, E2A, E2B, E3A, E3B, UP2, D2A, D2B, UP1, D1A, D1B, HEAD };

// Tensors a capture copies out, in this order: name, level (1: H x W,
// 2: H/2 x W/2, 3: H/4 x W/4) and channels.  Forward activations, then the
// stored output gradients (after the ReLU mask) in the order the backward
// pass makes them.
struct CapDef { const char *name; int level, ch; };
const CapDef kCap[] = {
    {"e1a", 1, 32}, {"e1b", 1, 32}, {"p1", 2, 32}, {"e2a", 2, 64}, {"e2b", 2, 64}, {"p2", 3, 64},
    {"e3a", 3, 128}, {"e3b", 3, 128}, {"up2", 2, 64}, {"d2a", 2, 64}, {"d2b", 2, 64}, {"up1", 1, 32},
    {"d1a", 1, 32}, {"d1b", 1, 32},
    {"dz_d1b", 1, 32}, {"dz_d1a", 1, 32}, {"dz_up1", 1, 32}, {"dz_d2b", 2, 64}, {"dz_d2a", 2, 64},
    {"dz_up2", 2, 64}, {"dz_e3b", 3, 128}, {"dz_e3a", 3, 128}, {"dz_e2b", 2, 64}, {"dz_e2a", 2, 64},
    {"dz_e1b", 1, 32}, {"dz_e1a", 1, 32}};
constexpr int kNCap = 26;
enum { C_DZ_D1B = 14 };

long long cap_elems(int idx, long long P)
{
    const int lv = kCap[idx].level;
    return (lv == 1 ? P : (lv == 2 ? P / 4 : P / 16)) * kCap[idx].ch;
}
long long cap_offset(int idx, long long P)
{
    long long o = 0;
    for (int i = 0; i < idx; ++i) o += cap_elems(i, P);
    return o;
}

int64_t wcount(const LayerDef &l)
{
    return l.kind == 0 ? 9LL * l.cin * l.cout : (l.kind == 1 ? 4LL * l.cin * l.cout : l.cin);
}
int64_t bcount(const LayerDef &l) { return l.kind == 2 ? 1 : l.cout; }

}  // namespace

struct lalm_unet {
    int Bmax = 0, H = 0, W = 0;
    int64_t woff[kNL], boff[kNL], nparam = 0;
    std::vector<void *> allocs;
    bf16 *wf[kNL] = {}, *wd[kNL] = {};
    // activations (bf16 NHWC)
    bf16 *e1a, *e1b, *p1, *e2a, *e2b, *p2, *e3a, *e3b, *up2, *d2a, *d2b, *up1, *d1a, *d1b;
    // gradient scratch
    float *gA, *gB, *gSkip1, *gSkip2, *dout, *part;
    bf16 *dzA, *dzB;
    double *lpart;
    int64_t part_elems = 0;
    const uint8_t *mask_ptr = nullptr;   // ROI mask whose pixel count is cached
    long long mask_count = 0;
};

namespace {

template <class T>
hipError_t alloc(lalm_unet *n, T **p, size_t count)
{
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) n->allocs.push_back((void *)*p);
    return e;
}

lalm_status ufail(lalm_status c, const std::string &m)
{
    lalm::set_error(m);
    return c;
}

#define UCHK(where, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return ufail(LALM_E_HIP, std::string(where) + ": " + hipGetErrorString(e_)); \
    } while (0)

// forward 3x3 conv (cin >= 32) at grid (B, h, w)
hipError_t conv_fwd(lalm_unet *n, int L, const bf16 *x1, int c1, const bf16 *x2, int c2, bf16 *y, const float *params,
                    int B, int h, int w, hipStream_t st, bf16 *pool = nullptr)
{
    GemmArgs g{};
    g.M = B * h * w;
    g.N = kLayers[L].cout;
    g.K = 9 * (c1 + c2);
    g.a1 = x1; g.a2 = x2; g.ac1 = c1; g.ac2 = c2;
    g.gB = B; g.gH = h; g.gW = w;
    g.ntap = 9; g.tsign = 1; g.ab = -1;
    g.w = n->wf[L];
    g.bias = params + n->boff[L];
    g.relu = 1;
    g.y = y;
    g.pool = pool;
    return conv3x3<E_FWD>(g, st, pool != nullptr);
}

hipError_t up_fwd(lalm_unet *n, int L, const bf16 *x, bf16 *y, const float *params, int B, int h, int w,
                  hipStream_t st)
{
    // the four output phases as one GEMM: the weights [phase][cout][cin]
    // are a (4 cout) x cin matrix, so the input is read once
    const int cin = kLayers[L].cin, cout = kLayers[L].cout;
    if (cout % 8) return hipErrorInvalidValue;
    GemmArgs g{};
    g.M = B * h * w;
    g.N = 4 * cout;
    g.K = cin;
    g.a1 = x; g.ac1 = cin;
    g.gB = B; g.gH = h; g.gW = w;
    g.ntap = 1; g.tsign = 1; g.ab = -1;
    g.w = n->wf[L];
    g.bias = params + n->boff[L];
    g.relu = 0;
    g.y = y; g.yup = 2; g.yc = cout;
    return gemm<A_CONV, B_W, E_FWD>(g, 1, st);
}

// Split-K weight-gradient GEMM (partials [split][M][N]) and the fixed-order
// reduction of the splits into dst.  Narrow outputs (M <= 32) take 32 x 128
// tiles; the split count fills the chip (about 2048 blocks) with at least 8
// K-tiles per split, within the partials buffer.
hipError_t wgrad_gemm(lalm_unet *n, GemmArgs &g, float *dst, hipStream_t st)
{
    const bool narrow = g.M <= 32;
    const int bm = narrow ? 32 : 64, bn = narrow ? 128 : 64;
    const int gx = (g.M + bm - 1) / bm, gy = (g.N + bn - 1) / bn;
    long long ns = (2048 + gx * gy - 1) / (gx * gy);
    ns = std::min<long long>(ns, std::max(1, g.K / (8 * BK)));
    ns = std::min<long long>(ns, n->part_elems / ((long long)g.M * g.N));
    ns = std::max<long long>(ns, 1);
    g.klen = (int)(((g.K + ns - 1) / ns + BK - 1) / BK * BK);
    ns = (g.K + g.klen - 1) / g.klen;
    g.part = n->part;
    const dim3 grd(gx, gy, (unsigned)ns);
    if (narrow) hipLaunchKernelGGL((wgrad_kernel<32, 128>), grd, dim3(256), 0, st, g);
    else hipLaunchKernelGGL((wgrad_kernel<64, 64>), grd, dim3(256), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long cnt = (long long)g.M * g.N;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(cnt, 32)), dim3(1024), 0, st, n->part, (int)ns, cnt, dst);
    return hipGetLastError();
}

// weight gradient of a 3x3 conv: dW[o][tap*cin + c] = sum_p dz[p][o] X[p+tap][c]
hipError_t conv_wgrad(lalm_unet *n, int L, const bf16 *dz, const bf16 *x1, int c1, const bf16 *x2, int c2,
                      float *grad, int B, int h, int w, hipStream_t st)
{
    GemmArgs g{};
    g.M = kLayers[L].cout;
    g.N = 9 * (c1 + c2);
    g.K = B * h * w;
    g.a1 = dz; g.ac1 = g.M; g.ab = -1;
    g.gB = B; g.gH = h; g.gW = w;
    g.b1 = x1; g.b2 = x2; g.bc1 = c1; g.bc2 = c2; g.bntap = 9;
    return wgrad_gemm(n, g, grad + n->woff[L], st);
}

hipError_t up_wgrad(lalm_unet *n, int L, const bf16 *dz_hi, const bf16 *x, float *grad, int B, int h, int w,
                    hipStream_t st)
{
    const int cin = kLayers[L].cin, cout = kLayers[L].cout;
    for (int ab = 0; ab < 4; ++ab) {
        GemmArgs g{};
        g.M = cout;
        g.N = cin;
        g.K = B * h * w;
        g.a1 = dz_hi; g.ac1 = cout; g.ab = ab;
        g.gB = B; g.gH = h; g.gW = w;
        g.b1 = x; g.bc1 = cin; g.bntap = 1;
        hipError_t e = wgrad_gemm(n, g, grad + n->woff[L] + (long long)ab * cout * cin, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// bias gradient: column sums of dz ([P][C] bf16)
hipError_t colsum(const bf16 *v, const float *mul, int C, long long P, int chunk, float *part, hipStream_t st)
{
    const unsigned ns = (unsigned)((P + chunk - 1) / chunk);
    if (C == 32) hipLaunchKernelGGL(colsum_kernel<32>, dim3(ns), dim3(256), 0, st, v, mul, P, chunk, part);
    else if (C == 64) hipLaunchKernelGGL(colsum_kernel<64>, dim3(ns), dim3(256), 0, st, v, mul, P, chunk, part);
    else if (C == 128) hipLaunchKernelGGL(colsum_kernel<128>, dim3(ns), dim3(256), 0, st, v, mul, P, chunk, part);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t bias_grad(lalm_unet *n, const bf16 *dz, int C, long long P, float *dst, hipStream_t st)
{
    const int chunk = 4096;
    const int ns = (int)((P + chunk - 1) / chunk);
    hipError_t e = colsum(dz, nullptr, C, P, chunk, n->part, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(C, 32)), dim3(1024), 0, st, n->part, ns, (long long)C, dst);
    return hipGetLastError();
}

// input gradient of a 3x3 conv: out[p][c] = sum_{tap, o} dz[p - tap][o] W[o][tap][c]
hipError_t conv_dgrad(lalm_unet *n, int L, const bf16 *dz, float *o1, int oc1, float *o2, int B, int h, int w,
                      hipStream_t st)
{
    GemmArgs g{};
    g.M = B * h * w;
    g.N = kLayers[L].cin;
    g.K = 9 * kLayers[L].cout;
    g.a1 = dz; g.ac1 = kLayers[L].cout; g.ac2 = 0;
    g.gB = B; g.gH = h; g.gW = w;
    g.ntap = 9; g.tsign = -1; g.ab = -1;
    g.w = n->wd[L];
    g.o1 = o1; g.o2 = o2; g.oc1 = oc1;
    return conv3x3<E_DG>(g, st);
}

// input gradient of a transposed conv: out[p][c] = sum_{ab, o} dz[up(p,ab)][o] W[ab][o][c]
hipError_t up_dgrad(lalm_unet *n, int L, const bf16 *dz_hi, float *out, int B, int h, int w, hipStream_t st)
{
    GemmArgs g{};
    g.M = B * h * w;
    g.N = kLayers[L].cin;
    g.K = 4 * kLayers[L].cout;
    g.a1 = dz_hi; g.ac1 = kLayers[L].cout;
    g.gB = B; g.gH = h; g.gW = w;
    g.ab = -1;
    g.w = n->wd[L];
    g.o1 = out; g.oc1 = g.N;
    return gemm<A_UPG, B_W, E_DG>(g, 1, st);
}

hipError_t to_dz(const float *gsrc, const bf16 *act, bf16 *dz, long long cnt, hipStream_t st)
{
    if (cnt % 8) return hipErrorInvalidValue;      // channel counts are multiples of 8
    hipLaunchKernelGGL(mask_to_bf16_kernel, dim3(nblk(cnt / 8)), dim3(256), 0, st, gsrc, act, dz, cnt / 8);
    return hipGetLastError();
}

lalm_status prep_weights(lalm_unet *n, const float *params, hipStream_t st)
{
    PrepTable T{};
    for (int L = 0; L < kNL; ++L) {
        const LayerDef &l = kLayers[L];
        if (!((l.kind == 0 && L != E1A) || l.kind == 1)) continue;
        if (T.n == kPrepMax) return ufail(LALM_E_STATE, "unet weights: too many layers");
        T.src[T.n] = params + n->woff[L];
        T.wf[T.n] = n->wf[L];
        T.wd[T.n] = n->wd[L];
        T.cout[T.n] = l.cout;
        T.cin[T.n] = l.cin;
        T.up[T.n] = l.kind == 1;
        T.start[T.n + 1] = T.start[T.n] + wcount(l);
        ++T.n;
    }
    hipLaunchKernelGGL(prep_all_kernel, dim3(nblk(T.start[T.n])), dim3(256), 0, st, T);
    UCHK("unet weights", hipGetLastError());
    return LALM_OK;
}

lalm_status run_forward(lalm_unet *n, const float *params, const float *x, float in_scale, int B, hipStream_t st)
{
    const int H = n->H, W = n->W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const long long P = (long long)B * H * W;
    lalm_status s = prep_weights(n, params, st);
    if (s != LALM_OK) return s;
    hipLaunchKernelGGL(conv1_mfma_kernel, dim3((unsigned)((P + 128 * C1_G - 1) / (128 * C1_G))), dim3(256), 0, st, x,
                       in_scale, params + n->woff[E1A], params + n->boff[E1A], n->e1a, B, H, W);
    UCHK("unet e1a", hipGetLastError());
    UCHK("unet e1b", conv_fwd(n, E1B, n->e1a, 32, nullptr, 0, n->e1b, params, B, H, W, st, n->p1));   // and p1
    UCHK("unet e2a", conv_fwd(n, E2A, n->p1, 32, nullptr, 0, n->e2a, params, B, H2, W2, st));
    UCHK("unet e2b", conv_fwd(n, E2B, n->e2a, 64, nullptr, 0, n->e2b, params, B, H2, W2, st));
    hipLaunchKernelGGL(pool_fwd_kernel, dim3(nblk(P / 16 * 64 / 8)), dim3(256), 0, st, n->e2b, n->p2, B, H2, W2, 64);
    UCHK("unet e3a", conv_fwd(n, E3A, n->p2, 64, nullptr, 0, n->e3a, params, B, H4, W4, st));
    UCHK("unet e3b", conv_fwd(n, E3B, n->e3a, 128, nullptr, 0, n->e3b, params, B, H4, W4, st));
    UCHK("unet up2", up_fwd(n, UP2, n->e3b, n->up2, params, B, H4, W4, st));
    UCHK("unet d2a", conv_fwd(n, D2A, n->up2, 64, n->e2b, 64, n->d2a, params, B, H2, W2, st));
    UCHK("unet d2b", conv_fwd(n, D2B, n->d2a, 64, nullptr, 0, n->d2b, params, B, H2, W2, st));
    UCHK("unet up1", up_fwd(n, UP1, n->d2b, n->up1, params, B, H2, W2, st));
    UCHK("unet d1a", conv_fwd(n, D1A, n->up1, 32, n->e1b, 32, n->d1a, params, B, H, W, st));
    UCHK("unet d1b", conv_fwd(n, D1B, n->d1a, 32, nullptr, 0, n->d1b, params, B, H, W, st));
    return LALM_OK;
}

}  // namespace

extern "C" int64_t lalm_unet_param_count(void)
{
    int64_t s = 0;
    for (int L = 0; L < kNL; ++L) s += wcount(kLayers[L]) + bcount(kLayers[L]);
    return s;
}

extern "C" lalm_status lalm_unet_create(int32_t batch_max, int32_t height, int32_t width, lalm_unet **out)
{
    if (!out) return ufail(LALM_E_INVALID, "lalm_unet_create: null argument");
    *out = nullptr;
    if (batch_max < 1 || height < 4 || width < 4 || height % 4 || width % 4)
        return ufail(LALM_E_INVALID, "lalm_unet_create: sizes must be positive multiples of 4");
    if ((long long)batch_max * height * width > (1LL << 30))
        return ufail(LALM_E_INVALID, "lalm_unet_create: batch too large");
    lalm_unet *n = new lalm_unet();
    n->Bmax = batch_max; n->H = height; n->W = width;
    int64_t o = 0;
    for (int L = 0; L < kNL; ++L) {
        n->woff[L] = o;
        o += wcount(kLayers[L]);
        n->boff[L] = o;
        o += bcount(kLayers[L]);
    }
    n->nparam = o;
    const long long P = (long long)batch_max * height * width, P2 = P / 4, P4 = P / 16;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    for (int L = 0; L < kNL; ++L) {
        if (kLayers[L].kind == 2 || L == E1A) continue;
        chk(alloc(n, &n->wf[L], (size_t)wcount(kLayers[L])));
        chk(alloc(n, &n->wd[L], (size_t)wcount(kLayers[L])));
    }
    chk(alloc(n, &n->e1a, P * 32)); chk(alloc(n, &n->e1b, P * 32)); chk(alloc(n, &n->p1, P2 * 32));
    chk(alloc(n, &n->e2a, P2 * 64)); chk(alloc(n, &n->e2b, P2 * 64)); chk(alloc(n, &n->p2, P4 * 64));
    chk(alloc(n, &n->e3a, P4 * 128)); chk(alloc(n, &n->e3b, P4 * 128)); chk(alloc(n, &n->up2, P2 * 64));
    chk(alloc(n, &n->d2a, P2 * 64)); chk(alloc(n, &n->d2b, P2 * 64)); chk(alloc(n, &n->up1, P * 32));
    chk(alloc(n, &n->d1a, P * 32)); chk(alloc(n, &n->d1b, P * 32));
    chk(alloc(n, &n->gA, P * 64)); chk(alloc(n, &n->gB, P * 64));
    chk(alloc(n, &n->gSkip1, P * 32)); chk(alloc(n, &n->gSkip2, P2 * 64));
    chk(alloc(n, &n->dout, P));
    chk(alloc(n, &n->dzA, P * 64)); chk(alloc(n, &n->dzB, P * 64));
    chk(alloc(n, &n->lpart, (size_t)(P / 256 + 1)));
    // partial sums: weight-gradient splits (the split count adapts to this
    // size) and per-chunk column sums
    n->part_elems = std::max<int64_t>(256LL * 128 * 1152, (P / 1024 + 1) * 320);
    chk(alloc(n, &n->part, (size_t)n->part_elems));
    if (e != hipSuccess) {
        std::string m = std::string("lalm_unet_create: allocation failed: ") + hipGetErrorString(e);
        lalm_unet_destroy(n);
        return ufail(LALM_E_NOMEM, m);
    }
    *out = n;
    return LALM_OK;
}

extern "C" lalm_status lalm_unet_destroy(lalm_unet *n)
{
    if (!n) return ufail(LALM_E_INVALID, "lalm_unet_destroy: null");
    (void)hipDeviceSynchronize();
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
    return LALM_OK;
}

extern "C" lalm_status lalm_unet_forward(lalm_unet *n, const float *params, const float *x, float *out,
                                         int32_t batch, double in_scale, int32_t nonneg, hipStream_t st)
{
    if (!n || !params || !x || !out) return ufail(LALM_E_INVALID, "lalm_unet_forward: null argument");
    if (batch < 1 || batch > n->Bmax) return ufail(LALM_E_INVALID, "lalm_unet_forward: batch out of range");
    if (!(in_scale > 0.0)) return ufail(LALM_E_INVALID, "lalm_unet_forward: in_scale must be positive");
    lalm_status s = run_forward(n, params, x, (float)in_scale, batch, st);
    if (s != LALM_OK) return s;
    const long long P = (long long)batch * n->H * n->W;
    hipLaunchKernelGGL(head_kernel, dim3(nblk(P)), dim3(256), 0, st, x, (float)(1.0 / in_scale), nonneg ? 1 : 0,
                       n->d1b, params + n->woff[HEAD], params + n->boff[HEAD], out, (const float *)nullptr,
                       (const uint8_t *)nullptr, 0.0, (float *)nullptr, (double *)nullptr, P, n->H * n->W);
    UCHK("unet head", hipGetLastError());
    return LALM_OK;
}

namespace {

// Loss, parameter gradient and, when cap is set, a copy of every stored
// tensor (FP32, in kCap order; see lalm_unet_capture).
lalm_status loss_grad_impl(lalm_unet *n, const float *params, const float *x, const float *target,
                           const uint8_t *mask, double in_scale, double hu_scale, int32_t batch, float *grad,
                           double *loss_dev, float *cap, hipStream_t st)
{
    if (!(in_scale > 0.0)) return ufail(LALM_E_INVALID, "lalm_unet_loss_grad: in_scale must be positive");
    if (!n || !params || !x || !target || !mask || !grad || !loss_dev)
        return ufail(LALM_E_INVALID, "lalm_unet_loss_grad: null argument");
    if (batch < 1 || batch > n->Bmax) return ufail(LALM_E_INVALID, "lalm_unet_loss_grad: batch out of range");
    if (mask != n->mask_ptr) {     // count the mask once per mask buffer
        std::vector<uint8_t> hm((size_t)n->H * n->W);
        UCHK("unet mask copy", hipMemcpyAsync(hm.data(), mask, hm.size(), hipMemcpyDeviceToHost, st));
        UCHK("unet mask sync", hipStreamSynchronize(st));
        long long cnt = 0;
        for (uint8_t v : hm) cnt += v ? 1 : 0;
        n->mask_ptr = mask;
        n->mask_count = cnt;
    }
    const long long nm = n->mask_count;
    if (nm == 0) return ufail(LALM_E_INVALID, "lalm_unet_loss_grad: empty mask");
    const int B = batch, H = n->H, W = n->W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const long long P = (long long)B * H * W, P2 = P / 4, P4 = P / 16;
    lalm_status s = run_forward(n, params, x, (float)in_scale, B, st);
    if (s != LALM_OK) return s;
    auto dump = [&](int idx, const bf16 *src) -> hipError_t {
        if (!cap) return hipSuccess;
        const long long cnt = cap_elems(idx, P);
        hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(nblk(cnt)), dim3(256), 0, st, src, cap + cap_offset(idx, P), cnt);
        return hipGetLastError();
    };
    const double s2n = hu_scale * hu_scale / (double)(nm * B);
    const unsigned hb = nblk(P);
    hipLaunchKernelGGL(head_kernel, dim3(hb), dim3(256), 0, st, x, (float)(1.0 / in_scale), 0, n->d1b,
                       params + n->woff[HEAD], params + n->boff[HEAD], (float *)nullptr, target, mask, s2n, n->dout,
                       n->lpart, P, H * W);
    hipLaunchKernelGGL(sum_double_kernel, dim3(1), dim3(256), 0, st, n->lpart, (int)hb, loss_dev);
    UCHK("unet loss", hipGetLastError());

    // head: weight gradient sum_p dout[p] d1b[p][c], bias sum_p dout[p]
    {
        const int chunk = 4096, ns = (int)((P + chunk - 1) / chunk);
        UCHK("head wgrad", colsum(n->d1b, n->dout, 32, P, chunk, n->part, st));
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, n->part, ns, 32LL, grad + n->woff[HEAD]);
        hipLaunchKernelGGL(sum_chunk_kernel, dim3(ns), dim3(256), 0, st, n->dout, P, chunk, n->part);
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(1024), 0, st, n->part, ns, 1LL, grad + n->boff[HEAD]);
        hipLaunchKernelGGL(head_bwd_kernel, dim3(nblk(P * 32)), dim3(256), 0, st, n->dout, n->d1b,
                           params + n->woff[HEAD], n->dzA, P);
        UCHK("unet head backward", hipGetLastError());
        UCHK("capture dz_d1b", dump(C_DZ_D1B, n->dzA));
    }
    bf16 *dz = n->dzA, *dz2 = n->dzB;
    // d1b: dz_d1b in dz
    UCHK("d1b wgrad", conv_wgrad(n, D1B, dz, n->d1a, 32, nullptr, 0, grad, B, H, W, st));
    UCHK("d1b bgrad", bias_grad(n, dz, 32, P, grad + n->boff[D1B], st));
    UCHK("d1b dgrad", conv_dgrad(n, D1B, dz, n->gA, 32, nullptr, B, H, W, st));
    UCHK("d1a dz", to_dz(n->gA, n->d1a, dz2, P * 32, st));
    std::swap(dz, dz2);
    UCHK("capture dz_d1a", dump(C_DZ_D1B + 1, dz));
    // d1a (input = concat[up1, e1b])
    UCHK("d1a wgrad", conv_wgrad(n, D1A, dz, n->up1, 32, n->e1b, 32, grad, B, H, W, st));
    UCHK("d1a bgrad", bias_grad(n, dz, 32, P, grad + n->boff[D1A], st));
    UCHK("d1a dgrad", conv_dgrad(n, D1A, dz, n->gA, 32, n->gSkip1, B, H, W, st));
    UCHK("up1 dz", to_dz(n->gA, nullptr, dz2, P * 32, st));
    std::swap(dz, dz2);
    UCHK("capture dz_up1", dump(C_DZ_D1B + 2, dz));
    // up1: input d2b at (H2, W2), output gradient dz at (H, W)
    UCHK("up1 wgrad", up_wgrad(n, UP1, dz, n->d2b, grad, B, H2, W2, st));
    UCHK("up1 bgrad", bias_grad(n, dz, 32, P, grad + n->boff[UP1], st));
    UCHK("up1 dgrad", up_dgrad(n, UP1, dz, n->gA, B, H2, W2, st));
    UCHK("d2b dz", to_dz(n->gA, n->d2b, dz2, P2 * 64, st));
    std::swap(dz, dz2);
    UCHK("capture dz_d2b", dump(C_DZ_D1B + 3, dz));
    UCHK("d2b wgrad", conv_wgrad(n, D2B, dz, n->d2a, 64, nullptr, 0, grad, B, H2, W2, st));
    UCHK("d2b bgrad", bias_grad(n, dz, 64, P2, grad + n->boff[D2B], st));
    UCHK("d2b dgrad", conv_dgrad(n, D2B, dz, n->gA, 64, nullptr, B, H2, W2, st));
    UCHK("d2a dz", to_dz(n->gA, n->d2a, dz2, P2 * 64, st));
    std::swap(dz, dz2);
    UCHK("capture dz_d2a", dump(C_DZ_D1B + 4, dz));
    UCHK("d2a wgrad", conv_wgrad(n, D2A, dz, n->up2, 64, n->e2b, 64, grad, B, H2, W2, st));
    UCHK("d2a bgrad", bias_grad(n, dz, 64, P2, grad + n->boff[D2A], st));
    UCHK("d2a dgrad", conv_dgrad(n, D2A, dz, n->gA, 64, n->gSkip2, B, H2, W2, st));
    UCHK("up2 dz", to_dz(n->gA, nullptr, dz2, P2 * 64, st));
    std::swap(dz, dz2);
    UCHK("capture dz_up2", dump(C_DZ_D1B + 5, dz));
    UCHK("up2 wgrad", up_wgrad(n, UP2, dz, n->e3b, grad, B, H4, W4, st));
    UCHK("up2 bgrad", bias_grad(n, dz, 64, P2, grad + n->boff[UP2], st));
    UCHK("up2 dgrad", up_dgrad(n, UP2, dz, n->gA, B, H4, W4, st));
    UCHK("e3b dz", to_dz(n->gA, n->e3b, dz2, P4 * 128, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e3b", dump(C_DZ_D1B + 6, dz));
    UCHK("e3b wgrad", conv_wgrad(n, E3B, dz, n->e3a, 128, nullptr, 0, grad, B, H4, W4, st));
    UCHK("e3b bgrad", bias_grad(n, dz, 128, P4, grad + n->boff[E3B], st));
    UCHK("e3b dgrad", conv_dgrad(n, E3B, dz, n->gA, 128, nullptr, B, H4, W4, st));
    UCHK("e3a dz", to_dz(n->gA, n->e3a, dz2, P4 * 128, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e3a", dump(C_DZ_D1B + 7, dz));
    UCHK("e3a wgrad", conv_wgrad(n, E3A, dz, n->p2, 64, nullptr, 0, grad, B, H4, W4, st));
    UCHK("e3a bgrad", bias_grad(n, dz, 128, P4, grad + n->boff[E3A], st));
    UCHK("e3a dgrad", conv_dgrad(n, E3A, dz, n->gA, 64, nullptr, B, H4, W4, st));
    // pool 2 backward into the skip gradient of e2b, then mask
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(nblk(P4 * 64)), dim3(256), 0, st, n->e2b, n->gA, n->gSkip2, B, H2, W2, 64);
    UCHK("pool2 backward", hipGetLastError());
    UCHK("e2b dz", to_dz(n->gSkip2, n->e2b, dz2, P2 * 64, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e2b", dump(C_DZ_D1B + 8, dz));
    UCHK("e2b wgrad", conv_wgrad(n, E2B, dz, n->e2a, 64, nullptr, 0, grad, B, H2, W2, st));
    UCHK("e2b bgrad", bias_grad(n, dz, 64, P2, grad + n->boff[E2B], st));
    UCHK("e2b dgrad", conv_dgrad(n, E2B, dz, n->gA, 64, nullptr, B, H2, W2, st));
    UCHK("e2a dz", to_dz(n->gA, n->e2a, dz2, P2 * 64, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e2a", dump(C_DZ_D1B + 9, dz));
    UCHK("e2a wgrad", conv_wgrad(n, E2A, dz, n->p1, 32, nullptr, 0, grad, B, H2, W2, st));
    UCHK("e2a bgrad", bias_grad(n, dz, 64, P2, grad + n->boff[E2A], st));
    UCHK("e2a dgrad", conv_dgrad(n, E2A, dz, n->gA, 32, nullptr, B, H2, W2, st));
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(nblk(P2 * 32)), dim3(256), 0, st, n->e1b, n->gA, n->gSkip1, B, H, W, 32);
    UCHK("pool1 backward", hipGetLastError());
    UCHK("e1b dz", to_dz(n->gSkip1, n->e1b, dz2, P * 32, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e1b", dump(C_DZ_D1B + 10, dz));
    UCHK("e1b wgrad", conv_wgrad(n, E1B, dz, n->e1a, 32, nullptr, 0, grad, B, H, W, st));
    UCHK("e1b bgrad", bias_grad(n, dz, 32, P, grad + n->boff[E1B], st));
    UCHK("e1b dgrad", conv_dgrad(n, E1B, dz, n->gA, 32, nullptr, B, H, W, st));
    UCHK("e1a dz", to_dz(n->gA, n->e1a, dz2, P * 32, st));
    std::swap(dz, dz2);
    UCHK("capture dz_e1a", dump(C_DZ_D1B + 11, dz));
    {
        // 1024 pixels per block: enough blocks to fill the chip at every batch size
        const int chunk = 1024, ns = (int)((P + chunk - 1) / chunk);
        hipLaunchKernelGGL(conv1_wgrad_kernel, dim3(ns), dim3(256), 0, st, x, (float)in_scale, dz, n->part, B, H, W,
                           chunk);
        // part[s][c*10 + t] -> weights [c][t] (t < 9) and bias [c]
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblk(320, 32)), dim3(1024), 0, st, n->part, ns, 320LL, n->gB);
        hipLaunchKernelGGL(scatter_conv1_kernel, dim3(1), dim3(320), 0, st, n->gB, grad + n->woff[E1A],
                           grad + n->boff[E1A]);
        UCHK("e1a wgrad", hipGetLastError());
    }
    if (cap) {
        const bf16 *acts[14] = {n->e1a, n->e1b, n->p1, n->e2a, n->e2b, n->p2, n->e3a,
                                n->e3b, n->up2, n->d2a, n->d2b, n->up1, n->d1a, n->d1b};
        for (int i = 0; i < 14; ++i) UCHK("capture activations", dump(i, acts[i]));
    }
    return LALM_OK;
}

}  // namespace

extern "C" lalm_status lalm_unet_loss_grad(lalm_unet *n, const float *params, const float *x, const float *target,
                                           const uint8_t *mask, double in_scale, double hu_scale, int32_t batch,
                                           float *grad, double *loss_dev, hipStream_t st)
{
    return loss_grad_impl(n, params, x, target, mask, in_scale, hu_scale, batch, grad, loss_dev, nullptr, st);
}

extern "C" int64_t lalm_unet_capture_elems(int32_t batch, int32_t height, int32_t width)
{
    if (batch < 1 || height < 4 || width < 4 || height % 4 || width % 4) return 0;
    const long long P = (long long)batch * height * width;
    return cap_offset(kNCap, P);
}

extern "C" lalm_status lalm_unet_capture(lalm_unet *n, const float *params, const float *x, const float *target,
                                         const uint8_t *mask, double in_scale, double hu_scale, int32_t batch,
                                         float *grad, double *loss_dev, float *capture, int64_t capture_elems,
                                         hipStream_t st)
{
    if (!n || !capture) return ufail(LALM_E_INVALID, "lalm_unet_capture: null argument");
    if (batch < 1 || batch > n->Bmax) return ufail(LALM_E_INVALID, "lalm_unet_capture: batch out of range");
    if (capture_elems < lalm_unet_capture_elems(batch, n->H, n->W))
        return ufail(LALM_E_INVALID, "lalm_unet_capture: capture buffer too small");
    return loss_grad_impl(n, params, x, target, mask, in_scale, hu_scale, batch, grad, loss_dev, capture, st);
}

extern "C" lalm_status lalm_unet_adam(lalm_unet *n, float *params, const float *grad, float *m, float *v, int64_t t,
                                      double lr, hipStream_t st)
{
    if (!n || !params || !grad || !m || !v || t < 1) return ufail(LALM_E_INVALID, "lalm_unet_adam: bad argument");
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(n->nparam)), dim3(256), 0, st, params, grad, m, v, (long long)n->nparam,
                       (float)lr, bc1, bc2);
    UCHK("unet adam", hipGetLastError());
    return LALM_OK;
}
