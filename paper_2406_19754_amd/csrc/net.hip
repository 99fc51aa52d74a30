// net.hip -- learned convolutional preconditioner for flexible CG on gfx950.
//
// Network (3 layers, 3x3x3 taps, 16 channels, zero padding, bias):
//   u = bf16(r / s), s = ||r|| / sqrt(N)
//   h1 = bf16(GELU(W1 * u + b1))           1 -> 16, FP32 vector FMA
//   h2 = bf16(GELU(W2 * h1 + b2))          16 -> 16, MFMA v_mfma_f32_16x16x32_bf16
//   out = W3 * h2 + b3,  z = s out         16 -> 1, FP32 vector FMA
// GELU(t) = t Phi(t). Activations are channel-last bfloat16 (32 bytes per
// cell), weights an FP32 master copy plus a bfloat16 working copy that is
// refreshed after every optimiser step.
//
// The 16 -> 16 layer is an implicit GEMM: one wavefront computes 16
// consecutive cells of an x-row times 16 output channels; the K dimension
// is (tap, input channel) = 27 x 16 = 432, covered by 14 MFMA steps of K=32
// (two taps per step, the last half empty). Lane l of the A operand holds
// the 8 input channels 8*((l>>4)&1).. of cell (l & 15) at tap 2t + (l>>5):
// one 16-byte load of the channel-last activations. The B operand (weights)
// is pre-arranged per step and lane once per weight update.
//
// Backward: the 16 -> 16 data gradient is the same MFMA kernel with the
// channel-transposed, tap-flipped weights; weight gradients are per-block
// FP32 partial sums over cells reduced in a fixed order (deterministic).
// Adam runs on the FP32 master copy.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/psc.h"
#include "kernels.h"
#include "net.h"

namespace psc {

extern thread_local std::string g_err;

static int nfail(int st, const std::string& m) {
    g_err = m;
    return st;
}

#define NHIPCHK(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return nfail(PSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int NC = 16;                       // channels
constexpr int NP = 7809;                     // parameters
constexpr int OW1 = 0, OB1 = 432, OW2 = 448, OB2 = 7360, OW3 = 7376, OB3 = 7808;
constexpr int KSTEPS = 14;                   // ceil(27 * 16 / 32) MFMA steps
constexpr int WGRAD_BLOCKS = 512;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16r;                // raw bfloat16 bits

// float -> bfloat16, round to nearest even (NaN kept quiet)
__host__ __device__ inline bf16r f2bf(float f) {
    unsigned u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        if (u & 0x007fffffu) u |= 0x00400000u;
        return (bf16r)(u >> 16);
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16r)(u >> 16);
}
__device__ inline float bf2f(bf16r b) { return __uint_as_float((unsigned)b << 16); }
// GELU(t) = t Phi(t) with Phi(t) = erfc(-t / sqrt 2) / 2, erfc(z) (z >= 0)
// from the Chebyshev fit erfc(z) = u exp(-z^2 + P(u)), u = 1 / (1 + z/2), of
// Press et al., Numerical Recipes (their erfcc; fractional error below
// 1.2e-7 for every z >= 0), evaluated branch-free in FP32 with the hardware
// reciprocal and exp2. In FP32 the result is within 5e-7 relative of the
// exact GELU for |t| <= 1, 2e-6 for -4 <= t <= -1 and 1.4e-7 for t >= 1;
// unlike 1 + erf(t / sqrt 2), it does not cancel for negative t.
__device__ inline float gelu(float t) {
    const float z = fabsf(t) * 0.70710678118654752f;
    const float u = __builtin_amdgcn_rcpf(fmaf(0.5f, z, 1.0f));
    float p = 0.17087277f;
    p = fmaf(p, u, -0.82215223f);
    p = fmaf(p, u, 1.48851587f);
    p = fmaf(p, u, -1.13520398f);
    p = fmaf(p, u, 0.27886807f);
    p = fmaf(p, u, -0.18628806f);
    p = fmaf(p, u, 0.09678418f);
    p = fmaf(p, u, 0.37409196f);
    p = fmaf(p, u, 1.00002368f);
    p = fmaf(p, u, -1.26551223f);
    const float e = u * __builtin_amdgcn_exp2f(fmaf(-z, z, p) * 1.44269504088896341f);   // erfc(z)
    const float phi = t >= 0.0f ? fmaf(-0.5f, e, 1.0f) : 0.5f * e;
    return t * phi;
}
// two floats to bfloat16 (round to nearest even), packed low then high
__device__ inline unsigned pack_bf16(float lo, float hi) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(unsigned, v);
}
__device__ inline float gelu_d(float t) {
    return 0.5f * (1.0f + erff(t * 0.70710678118654752f)) + t * expf(-0.5f * t * t) * 0.39894228040143268f;
}

// B samples of D x H x W cells (x fastest); cell c = ((b*D + z)*H + y)*W + x
struct Dims {
    int B, D, H, W;
    __host__ __device__ long long cells() const { return (long long)B * D * H * W; }
};

struct Cell {
    int b, z, y, x;
};
__device__ inline Cell cell_of(const Dims& d, long long c) {
    Cell r;
    r.x = (int)(c % d.W);
    long long t = c / d.W;
    r.y = (int)(t % d.H);
    t /= d.H;
    r.z = (int)(t % d.D);
    r.b = (int)(t / d.D);
    return r;
}
// neighbour at offset (dz-1, dy-1, dx-1) * sgn of tap t; -1 outside the sample
__device__ inline long long nbr(const Dims& d, const Cell& c, int t, int sgn) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int zz = c.z + sgn * dz, yy = c.y + sgn * dy, xx = c.x + sgn * dx;
    if (zz < 0 || zz >= d.D || yy < 0 || yy >= d.H || xx < 0 || xx >= d.W) return -1;
    return (((long long)c.b * d.D + zz) * d.H + yy) * d.W + xx;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// forward kernels
// ---------------------------------------------------------------------------

// u = bf16(r / s) (FP64 field, s = sqrt(*rr / N); s = 0 gives u = 0) or bf16(in).
template <bool FROM64>
__global__ __launch_bounds__(WG) void k_prep_u(long long n, const double* __restrict__ r64,
                                               const float* __restrict__ in32, const double* rr,
                                               long long N, bf16r* __restrict__ u, Gate g) {
    if (gate_skip(g)) return;
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= n) return;
    if (FROM64) {
        const double s = sqrt(*rr / (double)N);
        u[c] = s > 0.0 ? f2bf((float)(r64[c] / s)) : (bf16r)0;
    } else {
        u[c] = f2bf(in32[c]);
    }
}

// h1 = bf16(GELU(W1 * u + b1)); a1 = pre-activation (training only)
__global__ __launch_bounds__(WG) void k_conv1(Dims d, const bf16r* __restrict__ u, const float* __restrict__ wr,
                                              bf16r* __restrict__ h1, float* __restrict__ a1, Gate g) {
    if (gate_skip(g)) return;
    __shared__ float w[NC * 27 + NC];
    for (int i = threadIdx.x; i < NC * 27 + NC; i += WG) w[i] = wr[OW1 + i];
    __syncthreads();
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= d.cells()) return;
    const Cell cc = cell_of(d, c);
    float acc[NC];
#pragma unroll
    for (int co = 0; co < NC; co++) acc[co] = w[NC * 27 + co];
    for (int t = 0; t < 27; t++) {
        const long long nb = nbr(d, cc, t, 1);
        if (nb < 0) continue;
        const float v = bf2f(u[nb]);
#pragma unroll
        for (int co = 0; co < NC; co++) acc[co] += w[co * 27 + t] * v;
    }
    unsigned pk[NC / 2];
#pragma unroll
    for (int k = 0; k < NC / 2; k++)
        pk[k] = (unsigned)f2bf(gelu(acc[2 * k])) | ((unsigned)f2bf(gelu(acc[2 * k + 1])) << 16);
    u32x4* hp = (u32x4*)(h1 + c * NC);
    hp[0] = u32x4{pk[0], pk[1], pk[2], pk[3]};
    hp[1] = u32x4{pk[4], pk[5], pk[6], pk[7]};
    if (a1) {
        f32x4* ap = (f32x4*)(a1 + c * NC);
#pragma unroll
        for (int k = 0; k < 4; k++) ap[k] = f32x4{acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]};
    }
}

// 16 -> 16 convolution on MFMA. MODE 0 (forward): out = bias + W * in,
// aout = out (may be NULL), hout = bf16(GELU(out)). MODE 1 (data gradient
// with tap-flipped, channel-transposed weights): aout = (W' * in) * GELU'(aprev).
template <int MODE>
__global__ __launch_bounds__(WG) void k_conv2(Dims d, const bf16r* __restrict__ in,
                                              const bf16x8* __restrict__ frag, const float* __restrict__ wr,
                                              const float* __restrict__ aprev, float* __restrict__ aout,
                                              bf16r* __restrict__ hout, Gate g) {
    if (gate_skip(g)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tpr = (d.W + 15) / 16;
    const long long ntiles = (long long)d.B * d.D * d.H * tpr;
    const long long T = (long long)blockIdx.x * (WG / 64) + wv;
    if (T >= ntiles) return;   // uniform per wavefront
    const long long row = T / tpr;
    const int x0 = (int)(T % tpr) * 16;
    Cell cc;
    cc.y = (int)(row % d.H);
    cc.z = (int)((row / d.H) % d.D);
    cc.b = (int)(row / ((long long)d.H * d.D));
    cc.x = x0 + (lane & 15);
    const int half = (lane >> 4) & 1, tsel = lane >> 5;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int t = 0; t < KSTEPS; t++) {
        const int tap = 2 * t + tsel;
        u32x4 av = {0u, 0u, 0u, 0u};
        if (tap < 27 && cc.x < d.W) {
            const long long nb = nbr(d, cc, tap, 1);
            if (nb >= 0) av = *(const u32x4*)(in + nb * NC + half * 8);
        }
        const bf16x8 A = __builtin_bit_cast(bf16x8, av);
        const bf16x8 Bm = frag[t * 64 + lane];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bm, acc, 0, 0, 0);
    }
    // lane holds rows 4*(lane>>4)+i (cells) of column lane&15 (channel)
    const int co = lane & 15;
    const long long rowbase = row * d.W;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int xx = x0 + 4 * (lane >> 4) + i;
        if (xx >= d.W) continue;
        const long long c = rowbase + xx;
        float v = acc[i];
        if (MODE == 0) {
            v += wr[OB2 + co];
            if (aout) aout[c * NC + co] = v;
            hout[c * NC + co] = f2bf(gelu(v));
        } else {
            aout[c * NC + co] = v * gelu_d(aprev[c * NC + co]);
        }
    }
}

// Forward 16 -> 16 layer with the input tile staged in LDS: a workgroup
// computes 16 cells of 4 consecutive x-rows (one per wavefront) at one z; the
// 18 x 6 x 3 cells they read (zero outside the sample) are loaded once with
// 16-byte loads, and every MFMA step then takes its A operand from LDS
// instead of gathering it from the cache. Same operands and order as
// k_conv2<0>, so the same results.
constexpr int CT_X = 18, CT_Y = 6, CT_Z = 3, CT_CELLS = CT_X * CT_Y * CT_Z;
__global__ __launch_bounds__(WG) void k_conv2_lds(Dims d, const bf16r* __restrict__ in,
                                                  const bf16x8* __restrict__ frag, const float* __restrict__ wr,
                                                  float* __restrict__ aout, bf16r* __restrict__ hout, Gate g) {
    if (gate_skip(g)) return;
    __shared__ u32x4 tile[CT_CELLS * 2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nxt = (d.W + 15) / 16, nyt = (d.H + 3) / 4;
    long long t = blockIdx.x;
    const int x0 = (int)(t % nxt) * 16;
    t /= nxt;
    const int y0 = (int)(t % nyt) * 4;
    t /= nyt;
    const int z = (int)(t % d.D);
    const int b = (int)(t / d.D);
    for (int i = threadIdx.x; i < CT_CELLS * 2; i += WG) {
        const int cell = i >> 1, half = i & 1;
        const int rx = cell % CT_X, ry = (cell / CT_X) % CT_Y, rz = cell / (CT_X * CT_Y);
        const int xx = x0 + rx - 1, yy = y0 + ry - 1, zz = z + rz - 1;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (xx >= 0 && xx < d.W && yy >= 0 && yy < d.H && zz >= 0 && zz < d.D)
            v = *(const u32x4*)(in + ((((long long)b * d.D + zz) * d.H + yy) * d.W + xx) * NC + half * 8);
        tile[i] = v;
    }
    __syncthreads();
    const int y = y0 + wv;
    if (y >= d.H) return;   // uniform per wavefront; no barrier follows
    const int half = (lane >> 4) & 1, tsel = lane >> 5, cx = lane & 15;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int s = 0; s < KSTEPS; s++) {
        const int tap = 2 * s + tsel;
        u32x4 av = {0u, 0u, 0u, 0u};
        if (tap < 27) {
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // offsets + 1
            av = tile[(((dz * CT_Y) + wv + dy) * CT_X + cx + dx) * 2 + half];
        }
        const bf16x8 A = __builtin_bit_cast(bf16x8, av);
        const bf16x8 Bm = frag[s * 64 + lane];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bm, acc, 0, 0, 0);
    }
    const int co = lane & 15;
    const long long rowbase = (((long long)b * d.D + z) * d.H + y) * d.W;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int xx = x0 + 4 * (lane >> 4) + i;
        if (xx >= d.W) continue;
        const long long c = rowbase + xx;
        const float v = acc[i] + wr[OB2 + co];
        if (aout) aout[c * NC + co] = v;
        hout[c * NC + co] = f2bf(gelu(v));
    }
}

// out = W3 * h2 + b3; TO64: z = s * out with s = sqrt(*rr / N), else out32.
template <bool TO64>
__global__ __launch_bounds__(WG) void k_conv3(Dims d, const bf16r* __restrict__ h2, const float* __restrict__ wr,
                                              const double* rr, long long N, double* __restrict__ z64,
                                              float* __restrict__ out32, Gate g) {
    if (gate_skip(g)) return;
    __shared__ float w[NC * 27 + 1];
    for (int i = threadIdx.x; i < NC * 27 + 1; i += WG) w[i] = wr[OW3 + i];
    __syncthreads();
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= d.cells()) return;
    const Cell cc = cell_of(d, c);
    float acc = w[NC * 27];
    for (int t = 0; t < 27; t++) {
        const long long nb = nbr(d, cc, t, 1);
        if (nb < 0) continue;
        const u32x4* hp = (const u32x4*)(h2 + nb * NC);
        const u32x4 v0 = hp[0], v1 = hp[1];
        const unsigned pk[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
#pragma unroll
        for (int k = 0; k < 8; k++) {
            acc += w[(2 * k) * 27 + t] * __uint_as_float(pk[k] << 16);
            acc += w[(2 * k + 1) * 27 + t] * __uint_as_float(pk[k] & 0xffff0000u);
        }
    }
    if (TO64) {
        const double s = sqrt(*rr / (double)N);
        z64[c] = s * (double)acc;
    } else {
        out32[c] = acc;
    }
}

// ---------------------------------------------------------------------------
// fused inference: the three layers in one kernel
// ---------------------------------------------------------------------------
//
// One workgroup owns a 16 x 16 column of output cells in (x, y) and a range
// of z-planes, and walks it plane by plane, so that only r is read and z
// written in HBM (16 bytes per cell, plus the re-read halo of r). Output
// plane k-1 needs h2 on planes k-2..k over the 18 x 18 cells around the
// tile; h2 needs h1 on 20 x 20 cells and h1 needs u on 22 x 22. Step k
//   (1) stores u = bf16(r/s) of plane k+2 (22 x 22) in an LDS ring of three
//       planes (r was loaded into registers during step k-1);
//   (2) computes h1 on plane k+1 (20 x 20 cells) into an LDS ring of three
//       planes, channel-last in two 8-channel halves: per 16 cells one
//       16x16x32 MFMA, W1 (16 channels x 27 taps, padded to 32) as the A
//       operand and the cells' 27 input taps as the B operand;
//   (3) computes h2 on plane k (18 x 18 cells): the implicit GEMM of the
//       16 -> 16 layer (14 MFMA steps, K = (tap, channel)) with the weight
//       fragments as the A operand and the cells' neighbourhoods, read from
//       the h1 ring, as the B operand, so that a lane ends with four channels
//       of one cell; those registers are at once the B operand of two
//       16x16x16 MFMAs with W3 transposed (taps x channels), which give the 27
//       tap projections g_t(c) = sum_ch W3[ch][t] h2[ch](c) of every cell,
//       stored in LDS;
//   (4) adds for every output cell the projections g_t(c + offset_t) of the
//       9 taps with each dz to the plane they feed (k+1, k, k-1), kept in
//       three registers; plane k-1 is then complete: z = s (b3 + sum).
// Every convolution sums in FP32 (MFMA), activations are bfloat16 and zero
// outside the sample (the zero padding). Results equal the unfused kernels'
// up to FP32 summation order (which can move a bfloat16 rounding).
constexpr int FT = 16;                                       // output tile edge in x and y
constexpr int FE0 = FT + 6, FE1 = FT + 4, FE2 = FT + 2;      // u, h1, h2 region edges
constexpr int FN0 = FE0 * FE0, FN1 = FE1 * FE1, FN2 = FE2 * FE2;
constexpr int FT1 = (FN1 + 15) / 16, FT2 = (FN2 + 15) / 16;  // MFMA tiles of h1, h2
constexpr int FU_STRIDE = (FN0 + 7) & ~7;                    // bf16 elements per u plane
constexpr int FR_PER = (FN0 + WG - 1) / WG;                  // r values per thread and plane
// dynamic LDS, bytes: h1 ring u32x4[3][2][FN1] | projections float[27][FN2] | u ring bf16[3][FU_STRIDE]
constexpr int FL_H1 = 0;
constexpr int FL_G = FL_H1 + 3 * 2 * FN1 * 16;
constexpr int FL_U = FL_G + 27 * FN2 * 4;
constexpr int FL_BYTES = FL_U + 3 * FU_STRIDE * 2;
static_assert(FN1 % 16 == 0, "h1 region is whole MFMA tiles");
static_assert(FL_G % 16 == 0 && FL_U % 16 == 0, "LDS regions aligned");

typedef short s16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int ring3(int p) { return ((p % 3) + 3) % 3; }
__device__ __forceinline__ int slot3(int s0, int dz) { return s0 + dz >= 3 ? s0 + dz - 3 : s0 + dz; }
__device__ __forceinline__ unsigned wbits(float w) { return __float_as_uint(w) >> 16; }   // bf16-valued float

__global__ __launch_bounds__(WG) void k_net_fused(Dims d, int zc, const double* __restrict__ r, const double* rr,
                                                  long long N, const float* __restrict__ wr,
                                                  const bf16x8* __restrict__ frag, double* __restrict__ z, Gate g) {
    if (gate_skip(g)) return;
    extern __shared__ __align__(16) unsigned char fl[];
    u32x4* h1s = (u32x4*)(fl + FL_H1);
    float* gs = (float*)(fl + FL_G);
    bf16r* us = (bf16r*)(fl + FL_U);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n16 = lane & 15, grp = lane >> 4;
    const int ntx = (d.W + FT - 1) / FT, nty = (d.H + FT - 1) / FT;
    long long bid = blockIdx.x;
    const int x0 = (int)(bid % ntx) * FT;
    bid /= ntx;
    const int y0 = (int)(bid % nty) * FT;
    bid /= nty;
    const int z0 = (int)bid * zc;
    const int z1 = min(z0 + zc, d.D);
    const double s = sqrt(*rr / (double)N);
    const double s_inv = s > 0.0 ? 1.0 / s : 0.0;

    // weights of the working copy (bfloat16 values) as MFMA A operands
    bf16x8 w1f;   // W1[co = n16][tap 8 grp + j]
    {
        unsigned pk[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int t0 = 8 * grp + 2 * j, t1 = t0 + 1;
            const unsigned lo = t0 < 27 ? wbits(wr[OW1 + n16 * 27 + t0]) : 0u;
            const unsigned hi = t1 < 27 ? wbits(wr[OW1 + n16 * 27 + t1]) : 0u;
            pk[j] = lo | (hi << 16);
        }
        w1f = __builtin_bit_cast(bf16x8, u32x4{pk[0], pk[1], pk[2], pk[3]});
    }
    s16x4 w3f[2];   // W3[ch = 4 grp + i][tap = 16 m + n16]
#pragma unroll
    for (int m = 0; m < 2; m++) {
        const int t = 16 * m + n16;
        unsigned pk[2];
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int c0 = 4 * grp + 2 * j;
            const unsigned lo = t < 27 ? wbits(wr[OW3 + c0 * 27 + t]) : 0u;
            const unsigned hi = t < 27 ? wbits(wr[OW3 + (c0 + 1) * 27 + t]) : 0u;
            pk[j] = lo | (hi << 16);
        }
        w3f[m] = __builtin_bit_cast(s16x4, make_uint2(pk[0], pk[1]));
    }
    bf16x8 w2f[KSTEPS];
#pragma unroll
    for (int st = 0; st < KSTEPS; st++) w2f[st] = frag[st * 64 + lane];
    float b1v[4], b2v[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        b1v[i] = wr[OB1 + 4 * grp + i];
        b2v[i] = wr[OB2 + 4 * grp + i];
    }
    const float b3 = wr[OB3];
    // this lane's 8 layer-1 taps: offset in the u plane and dz (taps past 26
    // have zero weights; they read tap 26's input, which is finite)
    int t1off[8], t1dz[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int t = min(8 * grp + j, 26);
        t1dz[j] = t / 9;
        t1off[j] = ((t / 3) % 3) * FE0 + t % 3;
    }

    // r of plane p, cells tid + WG i of the 22 x 22 region, into registers
    double rv[FR_PER];
    auto load_r = [&](int p) {
#pragma unroll
        for (int i = 0; i < FR_PER; i++) {
            const int q = tid + WG * i;
            const int gx = x0 - 3 + q % FE0, gy = y0 - 3 + q / FE0;
            rv[i] = 0.0;
            if (q < FN0 && p >= 0 && p < d.D && gx >= 0 && gx < d.W && gy >= 0 && gy < d.H)
                rv[i] = r[((long long)p * d.H + gy) * d.W + gx];
        }
    };
    auto store_u = [&](int p) {
        bf16r* up = us + ring3(p) * FU_STRIDE;
#pragma unroll
        for (int i = 0; i < FR_PER; i++) {
            const int q = tid + WG * i;
            if (q < FN0) up[q] = f2bf((float)(rv[i] * s_inv));
        }
    };
    // (out-of-sample cells hold r = 0, so u = 0 there: the zero padding)
    load_r(z0 - 3);
    store_u(z0 - 3);
    load_r(z0 - 2);
    store_u(z0 - 2);
    load_r(z0 - 1);

    float oacc[3] = {0.f, 0.f, 0.f};   // output planes k-1, k, k+1
    const int ox = tid & 15, oy = tid >> 4;
    for (int k = z0 - 3; k <= z1; k++) {
        // (1) u of plane k+2; start loading r of plane k+3
        store_u(k + 2);
        load_r(k + 3);
        __syncthreads();
        // (2) h1 of plane k+1
        {
            const int p1 = k + 1;
            u32x4* h1p = h1s + ring3(p1) * 2 * FN1;
            const bool in1 = p1 >= 0 && p1 < d.D;
            const int s0 = ring3(p1 - 1);   // u slots of planes p1-1, p1, p1+1: s0, s0+1, s0+2 (mod 3)
            for (int T = wv; T < FT1; T += WG / 64) {
                const int q = T * 16 + n16;
                const int hx = q % FE1, hy = q / FE1;
                const int gx = x0 - 2 + hx, gy = y0 - 2 + hy;
                unsigned o0 = 0u, o1 = 0u;
                if (in1) {
                    unsigned pk[4];
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int ja = 2 * j, jb = 2 * j + 1;
                        const unsigned lo = us[slot3(s0, t1dz[ja]) * FU_STRIDE + hy * FE0 + hx + t1off[ja]];
                        const unsigned hi = us[slot3(s0, t1dz[jb]) * FU_STRIDE + hy * FE0 + hx + t1off[jb]];
                        pk[j] = lo | (hi << 16);
                    }
                    const bf16x8 B = __builtin_bit_cast(bf16x8, u32x4{pk[0], pk[1], pk[2], pk[3]});
                    const f32x4 a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f, B, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                    if (gx >= 0 && gx < d.W && gy >= 0 && gy < d.H) {
                        o0 = pack_bf16(gelu(a[0] + b1v[0]), gelu(a[1] + b1v[1]));
                        o1 = pack_bf16(gelu(a[2] + b1v[2]), gelu(a[3] + b1v[3]));
                    }
                }
                // channels 4 grp .. 4 grp + 3 of cell q
                uint2* dst = (uint2*)(h1p + (grp >> 1) * FN1 + q) + (grp & 1);
                *dst = make_uint2(o0, o1);
            }
        }
        __syncthreads();
        // (3) h2 of plane k and its tap projections
        const bool in2 = k >= z0 - 1 && k >= 0 && k < d.D;
        if (in2) {
            const int s0 = ring3(k - 1);   // h1 slots of planes k-1, k, k+1
            for (int T = wv; T < FT2; T += WG / 64) {
                const int q = T * 16 + n16;
                const bool valid = q < FN2;
                // cells past the region read cell 0 (their column of the product
                // is dropped); tap 27 (zero weights) reads tap 26's input
                const int ax = valid ? q % FE2 : 0, ay = valid ? q / FE2 : 0;
                const int gx = x0 - 1 + ax, gy = y0 - 1 + ay;
                const int base = ay * FE1 + ax + (grp & 1) * FN1;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int st = 0; st < KSTEPS; st++) {
                    const int tap = min(2 * st + (grp >> 1), 26);
                    const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
                    const u32x4 av = h1s[slot3(s0, dz) * 2 * FN1 + base + dy * FE1 + dx];
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[st], __builtin_bit_cast(bf16x8, av), acc, 0, 0, 0);
                }
                unsigned o0 = 0u, o1 = 0u;
                if (valid && gx >= 0 && gx < d.W && gy >= 0 && gy < d.H) {
                    o0 = pack_bf16(gelu(acc[0] + b2v[0]), gelu(acc[1] + b2v[1]));
                    o1 = pack_bf16(gelu(acc[2] + b2v[2]), gelu(acc[3] + b2v[3]));
                }
                const s16x4 hv = __builtin_bit_cast(s16x4, make_uint2(o0, o1));
                const f32x4 g0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3f[0], hv, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                const f32x4 g1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w3f[1], hv, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                if (valid) {
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        gs[(4 * grp + i) * FN2 + q] = g0[i];
                        const int t = 16 + 4 * grp + i;
                        if (t < 27) gs[t * FN2 + q] = g1[i];
                    }
                }
            }
        }
        __syncthreads();
        // (4) projections of plane k into output planes k+1 (dz = 0), k, k-1
        if (in2) {
#pragma unroll
            for (int dz = 0; dz < 3; dz++) {
                float sum = oacc[2 - dz];
#pragma unroll
                for (int dy = 0; dy < 3; dy++)
#pragma unroll
                    for (int dx = 0; dx < 3; dx++)
                        sum += gs[(dz * 9 + dy * 3 + dx) * FN2 + (oy + dy) * FE2 + ox + dx];
                oacc[2 - dz] = sum;
            }
        }
        const int pk1 = k - 1;
        if (pk1 >= z0 && pk1 < z1) {
            const int gx = x0 + ox, gy = y0 + oy;
            if (gx < d.W && gy < d.H) z[((long long)pk1 * d.H + gy) * d.W + gx] = s * (double)(b3 + oacc[0]);
        }
        oacc[0] = oacc[1];
        oacc[1] = oacc[2];
        oacc[2] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// loss and backward kernels
// ---------------------------------------------------------------------------

// g3 = 2 (out - target) / cnt on interior cells (0 elsewhere); partial sum of squares.
__global__ __launch_bounds__(WG) void k_loss(Dims d, int margin, double cnt, const float* __restrict__ out,
                                             const float* __restrict__ tgt, float* __restrict__ g3,
                                             double* __restrict__ part) {
    __shared__ double red[WG / 64];
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    double sq = 0.0;
    if (c < d.cells()) {
        const Cell cc = cell_of(d, c);
        const bool in = cc.z >= margin && cc.z < d.D - margin && cc.y >= margin && cc.y < d.H - margin &&
                        cc.x >= margin && cc.x < d.W - margin;
        const float df = in ? out[c] - tgt[c] : 0.0f;
        g3[c] = (float)(2.0 * (double)df / cnt);
        sq = (double)df * (double)df;
    }
    sq = wave_sum_d(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// sum of partials in a fixed order, times `scale`, into *dst
__global__ __launch_bounds__(WG) void k_sum_partials(const double* __restrict__ part, int n, double scale,
                                                     double* dst, float* dst32) {
    __shared__ double red[WG / 64];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += WG) a += part[i];
    a = wave_sum_d(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double s = ((red[0] + red[1]) + (red[2] + red[3])) * scale;
        if (dst) *dst = s;
        if (dst32) *dst32 = (float)s;
    }
}

// partial sums of r.r over blocks
__global__ __launch_bounds__(WG) void k_sumsq(long long n, const double* __restrict__ r, double* __restrict__ part) {
    __shared__ double red[WG / 64];
    double a = 0.0;
    for (long long i = (long long)blockIdx.x * WG + threadIdx.x; i < n; i += (long long)gridDim.x * WG)
        a += r[i] * r[i];
    a = wave_sum_d(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ga2 = (W3^T * g3) * GELU'(a2): FP32 copy (weight gradient) and bfloat16 copy (MFMA data gradient)
__global__ __launch_bounds__(WG) void k_conv3_bwd(Dims d, const float* __restrict__ g3, const float* __restrict__ wr,
                                                  const float* __restrict__ a2, float* __restrict__ ga2f,
                                                  bf16r* __restrict__ ga2b) {
    __shared__ float w[NC * 27];
    for (int i = threadIdx.x; i < NC * 27; i += WG) w[i] = wr[OW3 + i];
    __syncthreads();
    const long long c = (long long)blockIdx.x * WG + threadIdx.x;
    if (c >= d.cells()) return;
    const Cell cc = cell_of(d, c);
    float acc[NC];
#pragma unroll
    for (int ci = 0; ci < NC; ci++) acc[ci] = 0.f;
    for (int t = 0; t < 27; t++) {
        const long long nb = nbr(d, cc, t, -1);
        if (nb < 0) continue;
        const float gv = g3[nb];
#pragma unroll
        for (int ci = 0; ci < NC; ci++) acc[ci] += w[ci * 27 + t] * gv;
    }
    unsigned pk[NC / 2];
#pragma unroll
    for (int ci = 0; ci < NC; ci++) acc[ci] *= gelu_d(a2[c * NC + ci]);
#pragma unroll
    for (int k = 0; k < NC / 2; k++) pk[k] = (unsigned)f2bf(acc[2 * k]) | ((unsigned)f2bf(acc[2 * k + 1]) << 16);
    u32x4* hp = (u32x4*)(ga2b + c * NC);
    hp[0] = u32x4{pk[0], pk[1], pk[2], pk[3]};
    hp[1] = u32x4{pk[4], pk[5], pk[6], pk[7]};
    f32x4* ap = (f32x4*)(ga2f + c * NC);
#pragma unroll
    for (int k = 0; k < 4; k++) ap[k] = f32x4{acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]};
}

// Weight-gradient partials of one layer: dW[co][ci][t] = sum_c gout[c][co] in[c+off_t][ci],
// db[co] = sum_c gout[c][co]. Thread = (pair (co,ci), cell group); block = chunk of cells.
template <int CIN, int COUT>
__global__ __launch_bounds__(WG) void k_wgrad(Dims d, const bf16r* __restrict__ in, const float* __restrict__ gout,
                                              float* __restrict__ part) {
    constexpr int NPAIR = CIN * COUT, G = WG / NPAIR, NW = NPAIR * 27, STRIDE = NW + COUT;
    __shared__ float red[WG * 28];
    const int tid = threadIdx.x, pair = tid % NPAIR, grp = tid / NPAIR;
    const int co = pair / CIN, ci = pair % CIN;
    float acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = 0.f;
    float accb = 0.f;
    const long long n = d.cells();
    const long long per = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * per, hi = lo + per < n ? lo + per : n;
    if (grp < G) {
        for (long long c = lo + grp; c < hi; c += G) {
            const float gv = gout[c * COUT + co];
            const Cell cc = cell_of(d, c);
#pragma unroll
            for (int t = 0; t < 27; t++) {
                const long long nb = nbr(d, cc, t, 1);
                if (nb >= 0) acc[t] += gv * bf2f(in[nb * CIN + ci]);
            }
            accb += gv;
        }
    }
#pragma unroll
    for (int t = 0; t < 27; t++) red[tid * 28 + t] = acc[t];
    red[tid * 28 + 27] = accb;
    __syncthreads();
    if (tid < NPAIR) {
        float* dst = part + (size_t)blockIdx.x * STRIDE;
        for (int t = 0; t < 28; t++) {
            float s = 0.f;
            for (int g2 = 0; g2 < G; g2++) s += red[(g2 * NPAIR + tid) * 28 + t];
            if (t < 27) dst[tid * 27 + t] = s;
            else if (ci == 0) dst[NW + co] = s;
        }
    }
}

// Weight gradient of the 16 -> 16 layer on MFMA:
//   dW2[co][ci][t] = sum_c g[c][co] h1[c + off_t][ci],  db2[co] = sum_c g[c][co],
// an implicit GEMM per tap with the cells as the K dimension. A workgroup
// takes tiles of 4 x-rows x 32 cells at one z (wavefront w: row w); the tile's
// g (FP32, split into bfloat16 hi + lo so that the products keep about 16 bits)
// and the 6 x 3 rows x 34 cells of h1 it reaches (zero outside the sample)
// are staged in LDS channel-major, h1 in three copies shifted by dx so that
// every operand is one aligned 16-byte LDS read: lane l holds g of channel
// l & 15 at cells 8 (l >> 4) .. + 7 (A) and h1 of channel l & 15 at the same
// cells shifted by the tap (B). Each wavefront keeps the 27 tap accumulators
// (D[co = 4 (l >> 4) + i][ci = l & 15]) over the workgroup's tile range; the
// four wavefronts, then the blocks (k_wreduce), are added in a fixed order.
constexpr int WG2_X = 32, WG2_R = 4, WG2_HX = WG2_X + 2, WG2_HR = (WG2_R + 2) * 3;
__global__ __launch_bounds__(WG) void k_wgrad2_mfma(Dims d, const bf16r* __restrict__ h1, const float* __restrict__ g,
                                                    float* __restrict__ part) {
    __shared__ __align__(16) bf16r gl[2][WG2_R][NC][WG2_X];          // hi, lo
    __shared__ __align__(16) bf16r hl[3][WG2_HR][NC][WG2_X];         // shifted copies dx = 0, 1, 2
    __shared__ float red[WG / 64][NC * NC];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nxt = (d.W + WG2_X - 1) / WG2_X, nyt = (d.H + WG2_R - 1) / WG2_R;
    const long long ntiles = (long long)d.B * d.D * nyt * nxt;
    const long long per = (ntiles + gridDim.x - 1) / gridDim.x;
    const long long t0 = (long long)blockIdx.x * per, t1 = t0 + per < ntiles ? t0 + per : ntiles;
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) bacc[j] = 0.f;
    const int kg = lane >> 4, ch = lane & 15;
    for (long long T = t0; T < t1; T++) {
        long long q = T;
        const int x0 = (int)(q % nxt) * WG2_X;
        q /= nxt;
        const int y0 = (int)(q % nyt) * WG2_R;
        q /= nyt;
        const int z = (int)(q % d.D);
        const int b = (int)(q / d.D);
        __syncthreads();   // the previous tile's operands have been read
        {
            // g: 4 rows x 32 cells x 2 halves of 8 channels = 256 tasks
            const int cell = tid >> 1, half = tid & 1;
            const int r = cell / WG2_X, xi = cell % WG2_X;
            const int x = x0 + xi, y = y0 + r;
            float v[8];
            if (x < d.W && y < d.H) {
                const float* gp = g + ((((long long)b * d.D + z) * d.H + y) * d.W + x) * NC + half * 8;
                const f32x4 a = *(const f32x4*)gp, c = *(const f32x4*)(gp + 4);
                v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
                v[4] = c[0]; v[5] = c[1]; v[6] = c[2]; v[7] = c[3];
            } else {
#pragma unroll
                for (int j = 0; j < 8; j++) v[j] = 0.f;
            }
#pragma unroll
            for (int j = 0; j < 8; j++) {
                bacc[j] += v[j];
                const bf16r hi = f2bf(v[j]);
                const bf16r lo = f2bf(v[j] - __uint_as_float((unsigned)hi << 16));
                gl[0][r][half * 8 + j][xi] = hi;
                gl[1][r][half * 8 + j][xi] = lo;
            }
        }
        // h1: 18 rows x 34 cells x 2 halves
        for (int task = tid; task < WG2_HR * WG2_HX * 2; task += WG) {
            const int half = task & 1, cell = task >> 1;
            const int xi = cell % WG2_HX, row = cell / WG2_HX;
            const int dz = row / (WG2_R + 2), ry = row % (WG2_R + 2);
            const int x = x0 + xi - 1, y = y0 + ry - 1, zz = z + dz - 1;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (x >= 0 && x < d.W && y >= 0 && y < d.H && zz >= 0 && zz < d.D)
                v = *(const u32x4*)(h1 + ((((long long)b * d.D + zz) * d.H + y) * d.W + x) * NC + half * 8);
            const unsigned w[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
            for (int dx = 0; dx < 3; dx++) {
                const int pos = xi - dx;   // copy dx, position pos holds x0 + pos + dx - 1
                if (pos < 0 || pos >= WG2_X) continue;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    hl[dx][row][half * 8 + 2 * j][pos] = (bf16r)(w[j] & 0xffffu);
                    hl[dx][row][half * 8 + 2 * j + 1][pos] = (bf16r)(w[j] >> 16);
                }
            }
        }
        __syncthreads();
        const bf16x8 ahi = *(const bf16x8*)&gl[0][wv][ch][8 * kg];
        const bf16x8 alo = *(const bf16x8*)&gl[1][wv][ch][8 * kg];
#pragma unroll
        for (int t = 0; t < 27; t++) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const bf16x8 bm = *(const bf16x8*)&hl[dx][dz * (WG2_R + 2) + wv + dy][ch][8 * kg];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bm, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bm, acc[t], 0, 0, 0);
        }
    }
    // block partial: the four wavefronts' accumulators, tap by tap
    float* dst = part + (size_t)blockIdx.x * (NC * NC * 27 + NC);
    for (int t = 0; t < 27; t++) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; i++) red[wv][(4 * kg + i) * NC + ch] = acc[t][i];
        __syncthreads();
        // thread tid sums entry tid = co * 16 + ci over the wavefronts
        const float sum = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
        dst[tid * 27 + t] = sum;
    }
    // bias: threads with the same half hold the same 8 channels
    __syncthreads();
    float* bred = &red[0][0];   // 256 threads x 8 values would not fit: reduce in two rounds
    for (int j = 0; j < 8; j++) {
        __syncthreads();
        bred[tid] = bacc[j];
        __syncthreads();
        if (tid < 2) {
            float sum = 0.f;
            for (int k = tid; k < WG; k += 2) sum += bred[k];
            dst[NC * NC * 27 + tid * 8 + j] = sum;
        }
    }
}

// grad[ow + w] / grad[ob + co] = sum over blocks (fixed order) of the partials
__global__ __launch_bounds__(WG) void k_wreduce(const float* __restrict__ part, int nblk, int nw, int cout,
                                                int ow, int ob, float* __restrict__ grad) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= nw + cout) return;
    float s = 0.f;
    for (int b = 0; b < nblk; b++) s += part[(size_t)b * (nw + cout) + i];
    grad[i < nw ? ow + i : ob + (i - nw)] = s;
}

__global__ __launch_bounds__(WG) void k_adam(int np, float* __restrict__ p, float* __restrict__ m,
                                             float* __restrict__ v, const float* __restrict__ g, float lr,
                                             float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__device__ inline bool is_weight(int i) {
    return (i >= OW1 && i < OB1) || (i >= OW2 && i < OB2) || (i >= OW3 && i < OB3);
}

// Working copy: weights rounded to bfloat16 (held as float), biases FP32;
// MFMA B-operand fragments of W2 (forward) and of the tap-flipped,
// channel-transposed W2 (data gradient).
__global__ __launch_bounds__(WG) void k_refresh(const float* __restrict__ master, float* __restrict__ wr,
                                                bf16r* __restrict__ ffwd, bf16r* __restrict__ fbwd) {
    const int i = blockIdx.x * WG + threadIdx.x;
    if (i < NP) wr[i] = is_weight(i) ? __uint_as_float((unsigned)f2bf(master[i]) << 16) : master[i];
    if (i < KSTEPS * 64 * 8) {
        const int j = i & 7, l = (i >> 3) & 63, t = i >> 9;
        const int tap = 2 * t + (l >> 5);
        const int a = l & 15, bch = 8 * ((l >> 4) & 1) + j;
        bf16r vf = 0, vb = 0;
        if (tap < 27) {
            vf = f2bf(master[OW2 + (a * NC + bch) * 27 + tap]);          // W2[co=a][ci=bch][tap]
            vb = f2bf(master[OW2 + (bch * NC + a) * 27 + (26 - tap)]);   // W2[co=bch][ci=a][26-tap]
        }
        ffwd[i] = vf;
        fbwd[i] = vb;
    }
}

__global__ __launch_bounds__(WG) void k_gather(long long per, const float* __restrict__ src,
                                               const int* __restrict__ ids, int B, float* __restrict__ dst) {
    const long long t = (long long)blockIdx.x * WG + threadIdx.x;
    if (t >= per * B) return;
    const int b = (int)(t / per);
    dst[t] = src[(long long)ids[b] * per + (t % per)];
}

static inline unsigned blocks_for(long long n) { return (unsigned)((n + WG - 1) / WG); }

// Comparison arm of the learned form: one l1-Jacobi sweep from zero on the
// finest level, z = M_0^-1 r.
__global__ __launch_bounds__(WG) void k_jacobi_alt(long long n, const double* __restrict__ minv,
                                                   const double* __restrict__ r, double* __restrict__ z, Gate g) {
    if (gate_skip(g)) return;
    const long long i = (long long)blockIdx.x * WG + threadIdx.x;
    if (i < n) z[i] = minv[i] * r[i];
}

}  // namespace psc

using namespace psc;

struct psc_net {
    hipStream_t user_stream = nullptr, stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int device = 0;
    int kind = 0;                   // 0: the network; 1: l1-Jacobi alternate z = M_0^-1 r
    double* jminv = nullptr;        // kind 1: its own copy of M_0^-1
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *wr = nullptr;
    bf16r *ffwd = nullptr, *fbwd = nullptr;
    long long adam_t = 0;
    // inference grid
    int fused = 1;                  // 1: the fused 3-layer kernel; 0: one kernel per layer
    int gx = 0, gy = 0, gz = 0;
    long long gcells = 0;
    bf16r *u = nullptr, *h1 = nullptr, *h2 = nullptr;
    double* rr = nullptr;
    double* dpart = nullptr;        // 4096 doubles of reduction partials
    uint64_t gen = 1;
    // training buffers, sized for tcells cells
    long long tcells = 0;
    float *in_b = nullptr, *tgt_b = nullptr, *out_b = nullptr, *a1 = nullptr, *a2 = nullptr, *g3 = nullptr,
          *ga2f = nullptr, *ga1 = nullptr;
    bf16r *tu = nullptr, *th1 = nullptr, *th2 = nullptr, *ga2b = nullptr;
    double* lpart = nullptr;        // one loss partial per workgroup of the batch
    float* wpart = nullptr;
    double* loss_dev = nullptr;
};

namespace psc {

static void net_free_train(psc_net* n) {
    for (void* p : {(void*)n->in_b, (void*)n->tgt_b, (void*)n->out_b, (void*)n->a1, (void*)n->a2, (void*)n->g3,
                    (void*)n->ga2f, (void*)n->ga1, (void*)n->tu, (void*)n->th1, (void*)n->th2, (void*)n->ga2b,
                    (void*)n->lpart})
        if (p) (void)hipFree(p);
    n->in_b = n->tgt_b = n->out_b = n->a1 = n->a2 = n->g3 = n->ga2f = n->ga1 = nullptr;
    n->tu = n->th1 = n->th2 = n->ga2b = nullptr;
    n->lpart = nullptr;
    n->tcells = 0;
}

static int net_train_buffers(psc_net* n, long long cells) {
    if (cells <= n->tcells) return PSC_OK;
    NHIPCHK(hipStreamSynchronize(n->stream));
    net_free_train(n);
    const size_t c = (size_t)cells;
    NHIPCHK(hipMalloc(&n->in_b, c * 4));
    NHIPCHK(hipMalloc(&n->tgt_b, c * 4));
    NHIPCHK(hipMalloc(&n->out_b, c * 4));
    NHIPCHK(hipMalloc(&n->g3, c * 4));
    NHIPCHK(hipMalloc(&n->a1, c * NC * 4));
    NHIPCHK(hipMalloc(&n->a2, c * NC * 4));
    NHIPCHK(hipMalloc(&n->ga2f, c * NC * 4));
    NHIPCHK(hipMalloc(&n->ga1, c * NC * 4));
    NHIPCHK(hipMalloc(&n->tu, c * 2));
    NHIPCHK(hipMalloc(&n->th1, c * NC * 2));
    NHIPCHK(hipMalloc(&n->th2, c * NC * 2));
    NHIPCHK(hipMalloc(&n->ga2b, c * NC * 2));
    NHIPCHK(hipMalloc(&n->lpart, (c / WG + 2) * sizeof(double)));
    n->tcells = cells;
    return PSC_OK;
}

static void refresh(psc_net* n, hipStream_t st) {
    k_refresh<<<blocks_for(KSTEPS * 64 * 8 > NP ? KSTEPS * 64 * 8 : NP), WG, 0, st>>>(n->master, n->wr, n->ffwd, n->fbwd);
}

// Forward on B samples: input (FP64 r with *rr, or float in32) -> out.
static void forward(psc_net* n, hipStream_t st, const Dims& d, const double* r64, const float* in32,
                    const double* rr, long long N, bf16r* u, bf16r* h1, bf16r* h2, float* a1, float* a2,
                    double* z64, float* out32, Gate g) {
    const long long cells = d.cells();
    if (r64) k_prep_u<true><<<blocks_for(cells), WG, 0, st>>>(cells, r64, nullptr, rr, N, u, g);
    else k_prep_u<false><<<blocks_for(cells), WG, 0, st>>>(cells, nullptr, in32, nullptr, 1, u, g);
    k_conv1<<<blocks_for(cells), WG, 0, st>>>(d, u, n->wr, h1, a1, g);
    const long long tiles = (long long)d.B * d.D * ((d.H + 3) / 4) * ((d.W + 15) / 16);
    k_conv2_lds<<<(unsigned)tiles, WG, 0, st>>>(d, h1, (const bf16x8*)n->ffwd, n->wr, a2, h2, g);
    if (z64) k_conv3<true><<<blocks_for(cells), WG, 0, st>>>(d, h2, n->wr, rr, N, z64, nullptr, g);
    else k_conv3<false><<<blocks_for(cells), WG, 0, st>>>(d, h2, n->wr, nullptr, 1, nullptr, out32, g);
}

// z = s net(r/s) on one sample (d.B = 1) by the fused kernel: workgroups of
// 16 x 16 output columns, the z-range cut into chunks so that the grid has
// about 2048 workgroups (chunks of at least 8 planes).
static int fused_lds_ready(int dev) {
    static std::mutex mu;
    static bool done[64] = {};
    if (dev < 0 || dev >= 64) return nfail(PSC_ERR_ARG, "device ordinal beyond the fused-kernel table");
    std::lock_guard<std::mutex> lk(mu);
    if (!done[dev]) {
        if (FL_BYTES > 64 * 1024)
            NHIPCHK(hipFuncSetAttribute((const void*)k_net_fused, hipFuncAttributeMaxDynamicSharedMemorySize, FL_BYTES));
        done[dev] = true;
    }
    return PSC_OK;
}

static int forward_fused(psc_net* n, hipStream_t st, const Dims& d, const double* r64, const double* rr, long long N,
                         double* z64, Gate g) {
    int rc = fused_lds_ready(n->device);
    if (rc) return rc;
    const long long tiles = (long long)((d.W + FT - 1) / FT) * ((d.H + FT - 1) / FT);
    long long nch = (2048 + tiles - 1) / tiles;
    nch = std::max<long long>(1, std::min<long long>(nch, d.D / 8));
    const int zc = (int)((d.D + nch - 1) / nch);
    const long long blocks = tiles * ((d.D + zc - 1) / zc);
    k_net_fused<<<(unsigned)blocks, WG, FL_BYTES, st>>>(d, zc, r64, rr, N, n->wr, (const bf16x8*)n->ffwd, z64, g);
    return PSC_OK;
}

// Loss and gradient of the current batch (in_b, tgt_b) into n->grad; loss
// (mean) into *loss_dst (device double) and, if given, loss32 (device float).
static void loss_grad(psc_net* n, hipStream_t st, const Dims& d, int margin, double* loss_dst, float* loss32) {
    const long long cells = d.cells();
    const Gate g0{nullptr, GATE_NONE};
    forward(n, st, d, nullptr, n->in_b, nullptr, 1, n->tu, n->th1, n->th2, n->a1, n->a2, nullptr, n->out_b, g0);
    const double cnt = (double)d.B * (d.D - 2 * margin) * (d.H - 2 * margin) * (d.W - 2 * margin);
    const unsigned nb = blocks_for(cells);
    k_loss<<<nb, WG, 0, st>>>(d, margin, cnt, n->out_b, n->tgt_b, n->g3, n->lpart);
    k_sum_partials<<<1, WG, 0, st>>>(n->lpart, (int)nb, 1.0 / cnt, loss_dst, loss32);
    // layer 3: data gradient into ga2 and weight gradient
    k_conv3_bwd<<<nb, WG, 0, st>>>(d, n->g3, n->wr, n->a2, n->ga2f, n->ga2b);
    k_wgrad<NC, 1><<<WGRAD_BLOCKS, WG, 0, st>>>(d, n->th2, n->g3, n->wpart);
    k_wreduce<<<blocks_for(NC * 27 + 1), WG, 0, st>>>(n->wpart, WGRAD_BLOCKS, NC * 27, 1, OW3, OB3, n->grad);
    // layer 2: data gradient (MFMA) into ga1, weight gradient
    const long long tiles = (long long)d.B * d.D * d.H * ((d.W + 15) / 16);
    k_conv2<1><<<(unsigned)((tiles + 3) / 4), WG, 0, st>>>(d, n->ga2b, (const bf16x8*)n->fbwd, n->wr, n->a1, n->ga1,
                                                           nullptr, g0);
    k_wgrad2_mfma<<<WGRAD_BLOCKS, WG, 0, st>>>(d, n->th1, n->ga2f, n->wpart);
    k_wreduce<<<blocks_for(NC * NC * 27 + NC), WG, 0, st>>>(n->wpart, WGRAD_BLOCKS, NC * NC * 27, NC, OW2, OB2, n->grad);
    // layer 1: weight gradient
    k_wgrad<1, NC><<<WGRAD_BLOCKS, WG, 0, st>>>(d, n->tu, n->ga1, n->wpart);
    k_wreduce<<<blocks_for(NC * 27 + NC), WG, 0, st>>>(n->wpart, WGRAD_BLOCKS, NC * 27, NC, OW1, OB1, n->grad);
}

static int join_in(psc_net* n) {
    NHIPCHK(hipSetDevice(n->device));
    NHIPCHK(hipEventRecord(n->ev[0], n->user_stream));
    NHIPCHK(hipStreamWaitEvent(n->stream, n->ev[0], 0));
    return PSC_OK;
}
static int join_out(psc_net* n) {
    NHIPCHK(hipEventRecord(n->ev[1], n->stream));
    NHIPCHK(hipStreamWaitEvent(n->user_stream, n->ev[1], 0));
    return PSC_OK;
}

int net_launch_apply(psc_net* n, hipStream_t st, const double* r, double* z, const double* rr_dev, long long N,
                     Gate g) {
    if (!n || n->gcells != N) return nfail(PSC_ERR_ARG, "network grid does not match the vector size");
    if (n->kind == 1) {
        k_jacobi_alt<<<blocks_for(N), WG, 0, st>>>(N, n->jminv, r, z, g);
        return PSC_OK;
    }
    Dims d{1, n->gz, n->gy, n->gx};
    if (n->fused) return forward_fused(n, st, d, r, rr_dev, N, z, g);
    forward(n, st, d, r, nullptr, rr_dev, N, n->u, n->h1, n->h2, nullptr, nullptr, z, nullptr, g);
    return PSC_OK;
}

int net_check_grid(const psc_net* n, long long N) {
    if (!n) return nfail(PSC_ERR_ARG, "NULL network");
    if (n->gcells != N) return nfail(PSC_ERR_STATE, "psc_net_set_grid must give nx*ny*nz = n before a solve");
    return PSC_OK;
}

uint64_t net_generation(const psc_net* n) { return n ? n->gen : 0; }

}  // namespace psc

extern "C" {

int32_t psc_net_param_count(void) { return NP; }

void psc_net_free(psc_net* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    net_free_train(n);
    for (void* p : {(void*)n->master, (void*)n->m, (void*)n->v, (void*)n->grad, (void*)n->wr, (void*)n->ffwd,
                    (void*)n->fbwd, (void*)n->u, (void*)n->h1, (void*)n->h2, (void*)n->rr, (void*)n->dpart,
                    (void*)n->wpart, (void*)n->loss_dev, (void*)n->jminv})
        if (p) (void)hipFree(p);
    for (auto& e : n->ev)
        if (e) (void)hipEventDestroy(e);
    if (n->stream) (void)hipStreamDestroy(n->stream);
    delete n;
}

int psc_net_create(const float* params, void* hip_stream, psc_net** out) {
    if (!params || !out) return nfail(PSC_ERR_ARG, "NULL argument");
    *out = nullptr;
    psc_net* n = new psc_net();
    auto bail = [&](int st) { psc_net_free(n); return st; };
    n->user_stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&n->device) != hipSuccess) return bail(nfail(PSC_ERR_HIP, "hipGetDevice failed"));
    if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&n->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&n->ev[1], hipEventDisableTiming) != hipSuccess)
        return bail(nfail(PSC_ERR_HIP, "stream or event creation failed"));
    for (float** p : {&n->master, &n->m, &n->v, &n->grad, &n->wr})
        if (hipMalloc((void**)p, NP * sizeof(float)) != hipSuccess) return bail(nfail(PSC_ERR_OOM, "hipMalloc failed"));
    if (hipMalloc((void**)&n->ffwd, KSTEPS * 64 * 8 * 2) != hipSuccess ||
        hipMalloc((void**)&n->fbwd, KSTEPS * 64 * 8 * 2) != hipSuccess ||
        hipMalloc((void**)&n->rr, sizeof(double) * 2) != hipSuccess ||
        hipMalloc((void**)&n->dpart, sizeof(double) * 4096) != hipSuccess ||
        hipMalloc((void**)&n->loss_dev, sizeof(double) * 2) != hipSuccess ||
        hipMalloc((void**)&n->wpart, sizeof(float) * (size_t)WGRAD_BLOCKS * (NC * NC * 27 + NC)) != hipSuccess)
        return bail(nfail(PSC_ERR_OOM, "hipMalloc failed"));
    std::vector<float> zero(NP, 0.f);
    if (hipMemcpy(n->master, params, NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->m, zero.data(), NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->v, zero.data(), NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return bail(nfail(PSC_ERR_HIP, "parameter upload failed"));
    if (hipStreamSynchronize(n->user_stream) != hipSuccess) return bail(nfail(PSC_ERR_HIP, "stream sync failed"));
    refresh(n, n->stream);
    if (hipStreamSynchronize(n->stream) != hipSuccess) return bail(nfail(PSC_ERR_HIP, "weight refresh failed"));
    *out = n;
    return PSC_OK;
}

}  // extern "C"

namespace psc {
// An l1-Jacobi alternate for the learned schedule: its own device copy of
// the n entries of M_0^-1 (given in host memory), bound to hip_stream.
int net_create_jacobi(const double* minv_host, long long n, void* hip_stream, psc_net** out) {
    *out = nullptr;
    psc_net* net = new psc_net();
    auto bail = [&](int st) { psc_net_free(net); return st; };
    net->kind = 1;
    net->user_stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&net->device) != hipSuccess) return bail(nfail(PSC_ERR_HIP, "hipGetDevice failed"));
    if (hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&net->ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&net->ev[1], hipEventDisableTiming) != hipSuccess)
        return bail(nfail(PSC_ERR_HIP, "stream or event creation failed"));
    if (hipMalloc((void**)&net->jminv, (size_t)n * sizeof(double)) != hipSuccess)
        return bail(nfail(PSC_ERR_OOM, "hipMalloc failed"));
    if (hipMemcpy(net->jminv, minv_host, (size_t)n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return bail(nfail(PSC_ERR_HIP, "copy of M_0^-1 failed"));
    net->gx = (int)n;
    net->gy = net->gz = 1;
    net->gcells = n;
    *out = net;
    return PSC_OK;
}
}  // namespace psc

extern "C" {

int psc_net_get_params(const psc_net* n, float* params) {
    if (!n || !params) return nfail(PSC_ERR_ARG, "NULL argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    NHIPCHK(hipSetDevice(n->device));
    NHIPCHK(hipStreamSynchronize(n->stream));
    NHIPCHK(hipMemcpy(params, n->master, NP * sizeof(float), hipMemcpyDeviceToHost));
    return PSC_OK;
}

int psc_net_set_params(psc_net* n, const float* params) {
    if (!n || !params) return nfail(PSC_ERR_ARG, "NULL argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    int st = join_in(n);
    if (st) return st;
    NHIPCHK(hipMemcpyAsync(n->master, params, NP * sizeof(float), hipMemcpyHostToDevice, n->stream));
    NHIPCHK(hipMemsetAsync(n->m, 0, NP * sizeof(float), n->stream));
    NHIPCHK(hipMemsetAsync(n->v, 0, NP * sizeof(float), n->stream));
    n->adam_t = 0;
    refresh(n, n->stream);
    NHIPCHK(hipStreamSynchronize(n->stream));
    return join_out(n);
}

}  // extern "C"

namespace psc {
// The per-layer activations of the unfused inference kernels (u, h1, h2) for
// `cells` cells; none with the fused kernel. Bumps the generation, so that
// captured solver iterations are captured again.
static int grid_buffers(psc_net* n, long long cells) {
    for (bf16r** p : {&n->u, &n->h1, &n->h2})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    n->gen += 1;
    if (n->fused || cells == 0) return PSC_OK;
    NHIPCHK(hipMalloc((void**)&n->u, (size_t)cells * 2));
    NHIPCHK(hipMalloc((void**)&n->h1, (size_t)cells * NC * 2));
    NHIPCHK(hipMalloc((void**)&n->h2, (size_t)cells * NC * 2));
    return PSC_OK;
}
}  // namespace psc

extern "C" {

int psc_net_set_grid(psc_net* n, int32_t nx, int32_t ny, int32_t nz) {
    if (!n || nx < 1 || ny < 1 || nz < 1) return nfail(PSC_ERR_ARG, "bad grid");
    const long long cells = (long long)nx * ny * nz;
    if (n->kind == 1) {
        if (cells != n->gcells) return nfail(PSC_ERR_ARG, "an l1-Jacobi alternate acts on its matrix's rows only");
        return PSC_OK;
    }
    if (n->gx == nx && n->gy == ny && n->gz == nz) return PSC_OK;
    NHIPCHK(hipSetDevice(n->device));
    NHIPCHK(hipStreamSynchronize(n->stream));
    n->gx = n->gy = n->gz = 0;
    n->gcells = 0;
    const int st = grid_buffers(n, cells);
    if (st) return st;
    n->gx = nx;
    n->gy = ny;
    n->gz = nz;
    n->gcells = cells;
    return PSC_OK;
}

int psc_net_tune(psc_net* n, int32_t key, int32_t value) {
    if (!n) return nfail(PSC_ERR_ARG, "NULL network");
    if (key != PSC_NET_TUNE_FUSED) return nfail(PSC_ERR_ARG, "unknown network tuning key");
    if (n->kind != 0) return PSC_OK;   // the l1-Jacobi alternate has no layers
    const int f = value != 0;
    if (f == n->fused) return PSC_OK;
    NHIPCHK(hipSetDevice(n->device));
    NHIPCHK(hipStreamSynchronize(n->stream));
    n->fused = f;
    return grid_buffers(n, n->gcells);
}

int psc_net_apply(psc_net* n, const double* r, double* z, int32_t nx, int32_t ny, int32_t nz) {
    if (!n || !r || !z) return nfail(PSC_ERR_ARG, "NULL argument");
    int st = psc_net_set_grid(n, nx, ny, nz);
    if (st) return st;
    st = join_in(n);
    if (st) return st;
    const long long N = n->gcells;
    if (n->kind == 1) {
        net_launch_apply(n, n->stream, r, z, nullptr, N, Gate{nullptr, GATE_NONE});
        NHIPCHK(hipGetLastError());
        NHIPCHK(hipStreamSynchronize(n->stream));
        return join_out(n);
    }
    const unsigned nb = 1024;
    k_sumsq<<<nb, WG, 0, n->stream>>>(N, r, n->dpart);
    k_sum_partials<<<1, WG, 0, n->stream>>>(n->dpart, (int)nb, 1.0, n->rr, nullptr);
    st = net_launch_apply(n, n->stream, r, z, n->rr, N, Gate{nullptr, GATE_NONE});
    if (st) return st;
    NHIPCHK(hipGetLastError());
    NHIPCHK(hipStreamSynchronize(n->stream));
    return join_out(n);
}

int psc_net_forward_batch(psc_net* n, const float* in, float* out, int32_t B, int32_t D) {
    if (!n || !in || !out || B < 1 || D < 1) return nfail(PSC_ERR_ARG, "bad argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    Dims d{B, D, D, D};
    int st = join_in(n);
    if (st) return st;
    st = net_train_buffers(n, d.cells());
    if (st) return st;
    forward(n, n->stream, d, nullptr, in, nullptr, 1, n->tu, n->th1, n->th2, nullptr, nullptr, nullptr, out,
            Gate{nullptr, GATE_NONE});
    NHIPCHK(hipGetLastError());
    NHIPCHK(hipStreamSynchronize(n->stream));
    return join_out(n);
}

int psc_net_loss_grad(psc_net* n, const float* in, const float* tgt, int32_t B, int32_t D, int32_t margin,
                      float* loss, float* grad_host) {
    if (!n || !in || !tgt || !loss || !grad_host || B < 1 || D < 1 || margin < 0 || 2 * margin >= D)
        return nfail(PSC_ERR_ARG, "bad argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    Dims d{B, D, D, D};
    int st = join_in(n);
    if (st) return st;
    st = net_train_buffers(n, d.cells());
    if (st) return st;
    const size_t bytes = (size_t)d.cells() * 4;
    NHIPCHK(hipMemcpyAsync(n->in_b, in, bytes, hipMemcpyDeviceToDevice, n->stream));
    NHIPCHK(hipMemcpyAsync(n->tgt_b, tgt, bytes, hipMemcpyDeviceToDevice, n->stream));
    loss_grad(n, n->stream, d, margin, n->loss_dev, nullptr);
    NHIPCHK(hipGetLastError());
    double l = 0.0;
    NHIPCHK(hipMemcpyAsync(&l, n->loss_dev, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    NHIPCHK(hipMemcpyAsync(grad_host, n->grad, NP * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIPCHK(hipStreamSynchronize(n->stream));
    *loss = (float)l;
    return join_out(n);
}

int psc_net_train(psc_net* n, const float* r_crops, const float* z_crops, int32_t ncrops, int32_t crop,
                  int32_t margin, const int32_t* order, int32_t steps, int32_t batch, float lr, float beta1,
                  float beta2, float eps, float* losses_host) {
    if (!n || !r_crops || !z_crops || !order || ncrops < 1 || crop < 1 || steps < 0 || batch < 1 ||
        margin < 0 || 2 * margin >= crop || !(lr > 0.f))
        return nfail(PSC_ERR_ARG, "bad argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    for (long long i = 0; i < (long long)steps * batch; i++)
        if (order[i] < 0 || order[i] >= ncrops) return nfail(PSC_ERR_ARG, "crop index out of range");
    Dims d{batch, crop, crop, crop};
    int st = join_in(n);
    if (st) return st;
    st = net_train_buffers(n, d.cells());
    if (st) return st;
    int* ids = nullptr;
    float* ldev = nullptr;
    NHIPCHK(hipMalloc((void**)&ids, sizeof(int) * (size_t)steps * batch + 4));
    NHIPCHK(hipMalloc((void**)&ldev, sizeof(float) * (size_t)steps + 4));
    NHIPCHK(hipMemcpyAsync(ids, order, sizeof(int) * (size_t)steps * batch, hipMemcpyHostToDevice, n->stream));
    const long long per = (long long)crop * crop * crop;
    for (int s = 0; s < steps; s++) {
        k_gather<<<blocks_for(per * batch), WG, 0, n->stream>>>(per, r_crops, ids + (size_t)s * batch, batch, n->in_b);
        k_gather<<<blocks_for(per * batch), WG, 0, n->stream>>>(per, z_crops, ids + (size_t)s * batch, batch, n->tgt_b);
        loss_grad(n, n->stream, d, margin, n->loss_dev, ldev + s);
        n->adam_t += 1;
        const float c1 = 1.f - powf(beta1, (float)n->adam_t), c2 = 1.f - powf(beta2, (float)n->adam_t);
        k_adam<<<blocks_for(NP), WG, 0, n->stream>>>(NP, n->master, n->m, n->v, n->grad, lr, beta1, beta2, eps, c1, c2);
        refresh(n, n->stream);
    }
    NHIPCHK(hipGetLastError());
    if (losses_host && steps > 0)
        NHIPCHK(hipMemcpyAsync(losses_host, ldev, sizeof(float) * steps, hipMemcpyDeviceToHost, n->stream));
    NHIPCHK(hipStreamSynchronize(n->stream));
    (void)hipFree(ids);
    (void)hipFree(ldev);
    return join_out(n);
}


// ---- allocation-free apply ------------------------------------------------
// psc_net_apply_noalloc keeps its scratch (the ||r||^2 partials and sum, and
// the three bfloat16 activation fields) in one file-scope device array of
// fixed size instead of buffers sized per grid. Each device holds its own copy
// until the process ends; its address is looked up once per device and the
// kernels receive that address, never the host-side symbol. Layout (bytes):
//   [0, 16) ||r||^2 | [256, 256 + 8*NA_PARTS) partials | h1 | h2 | u
// with h1, h2 sized 32 bytes and u 2 bytes per cell of the largest grid.
constexpr int NA_PARTS = 1024;
constexpr long long NA_H1 = 256 + 8 * NA_PARTS;
constexpr long long NA_H2 = NA_H1 + 32ll * PSC_NET_NOALLOC_MAX_CELLS;
constexpr long long NA_U = NA_H2 + 32ll * PSC_NET_NOALLOC_MAX_CELLS;
constexpr long long NA_BYTES = NA_U + 2ll * PSC_NET_NOALLOC_MAX_CELLS;
static_assert(NA_H1 % 256 == 0 && NA_H2 % 256 == 0 && NA_U % 256 == 0, "scratch regions stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_dev[NA_MAX_DEVICES] = {};

// Device address of `scratch` on `dev` (which must be current), looked up on
// the first call for that device.
static int scratch_on(int dev, unsigned char** out) {
    if (dev < 0 || dev >= NA_MAX_DEVICES) return nfail(PSC_ERR_ARG, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return nfail(PSC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned char*)ptr;
    }
    *out = g_scratch_dev[dev];
    return PSC_OK;
}

int psc_net_apply_noalloc(psc_net* n, const double* r, double* z, int32_t nx, int32_t ny, int32_t nz) {
    if (!n || !r || !z) return nfail(PSC_ERR_ARG, "NULL argument");
    if (nx < 1 || ny < 1 || nz < 1) return nfail(PSC_ERR_ARG, "bad grid");
    const long long N = (long long)nx * ny * nz;
    if (N > PSC_NET_NOALLOC_MAX_CELLS)
        return nfail(PSC_ERR_ARG, "grid of " + std::to_string(N) + " cells exceeds the allocation-free maximum of " +
                                      std::to_string(PSC_NET_NOALLOC_MAX_CELLS) + " cells");
    NHIPCHK(hipSetDevice(n->device));
    if (n->kind == 1) {
        if (N != n->gcells) return nfail(PSC_ERR_ARG, "an l1-Jacobi alternate acts on its matrix's rows only");
        int sj = join_in(n);
        if (sj) return sj;
        k_jacobi_alt<<<blocks_for(N), WG, 0, n->stream>>>(N, n->jminv, r, z, Gate{nullptr, GATE_NONE});
        NHIPCHK(hipGetLastError());
        NHIPCHK(hipStreamSynchronize(n->stream));
        return join_out(n);
    }
    unsigned char* base = nullptr;
    int st = scratch_on(n->device, &base);
    if (st) return st;
    st = join_in(n);
    if (st) return st;
    double* rr = (double*)base;
    double* part = (double*)(base + 256);
    bf16r* h1 = (bf16r*)(base + NA_H1);
    bf16r* h2 = (bf16r*)(base + NA_H2);
    bf16r* u = (bf16r*)(base + NA_U);
    k_sumsq<<<NA_PARTS, WG, 0, n->stream>>>(N, r, part);
    k_sum_partials<<<1, WG, 0, n->stream>>>(part, NA_PARTS, 1.0, rr, nullptr);
    const Dims d{1, nz, ny, nx};
    if (n->fused) {
        st = forward_fused(n, n->stream, d, r, rr, N, z, Gate{nullptr, GATE_NONE});
        if (st) return st;
    } else {
        forward(n, n->stream, d, r, nullptr, rr, N, u, h1, h2, nullptr, nullptr, z, nullptr, Gate{nullptr, GATE_NONE});
    }
    NHIPCHK(hipGetLastError());
    NHIPCHK(hipStreamSynchronize(n->stream));
    return join_out(n);
}

// Checkpoint file: a 40-byte little-endian header, then the FP32 master
// weights, then (flag bit 0) the two Adam moment vectors, each param-count
// floats in the order of psc_net_get_params.
static const char kMagic[8] = {'P', 'S', 'C', 'N', 'E', 'T', '0', '1'};
struct NetFileHeader {
    char magic[8];
    uint32_t header_bytes, nparams, channels, ksize, flags, reserved;
    int64_t adam_t;
};
static_assert(sizeof(NetFileHeader) == 40, "checkpoint header layout");

static bool host_little_endian() {
    const uint32_t one = 1;
    unsigned char c;
    std::memcpy(&c, &one, 1);
    return c == 1;
}

int psc_net_save(const psc_net* n, const char* path) {
    if (!n || !path) return nfail(PSC_ERR_ARG, "NULL argument");
    if (n->kind != 0) return nfail(PSC_ERR_STATE, "an l1-Jacobi alternate has no weights");
    if (!host_little_endian()) return nfail(PSC_ERR_IO, "checkpoints are little-endian; host is not");
    std::vector<float> buf((size_t)3 * NP);
    NHIPCHK(hipSetDevice(n->device));
    NHIPCHK(hipStreamSynchronize(n->stream));
    NHIPCHK(hipMemcpy(buf.data(), n->master, NP * sizeof(float), hipMemcpyDeviceToHost));
    NHIPCHK(hipMemcpy(buf.data() + NP, n->m, NP * sizeof(float), hipMemcpyDeviceToHost));
    NHIPCHK(hipMemcpy(buf.data() + 2 * NP, n->v, NP * sizeof(float), hipMemcpyDeviceToHost));
    NetFileHeader hd{};
    std::memcpy(hd.magic, kMagic, 8);
    hd.header_bytes = sizeof(NetFileHeader);
    hd.nparams = NP;
    hd.channels = NC;
    hd.ksize = 3;
    hd.flags = 1;
    hd.adam_t = n->adam_t;
    FILE* f = std::fopen(path, "wb");
    if (!f) return nfail(PSC_ERR_IO, std::string("cannot open for writing: ") + path);
    bool ok = std::fwrite(&hd, sizeof hd, 1, f) == 1 && std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return nfail(PSC_ERR_IO, std::string("write failed: ") + path);
    return PSC_OK;
}

int psc_net_load(const char* path, void* hip_stream, psc_net** out) {
    if (!path || !out) return nfail(PSC_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (!host_little_endian()) return nfail(PSC_ERR_IO, "checkpoints are little-endian; host is not");
    FILE* f = std::fopen(path, "rb");
    if (!f) return nfail(PSC_ERR_IO, std::string("cannot open for reading: ") + path);
    NetFileHeader hd{};
    std::vector<float> buf((size_t)3 * NP, 0.f);
    bool ok = std::fread(&hd, sizeof hd, 1, f) == 1;
    std::string why;
    if (!ok) why = "short header";
    else if (std::memcmp(hd.magic, kMagic, 8) != 0) why = "not a network checkpoint (bad magic)";
    else if (hd.header_bytes != sizeof(NetFileHeader) || hd.nparams != (uint32_t)NP || hd.channels != (uint32_t)NC ||
             hd.ksize != 3 || (hd.flags & ~1u) != 0 || hd.adam_t < 0)
        why = "checkpoint header does not match this network (size, channels, kernel or flags)";
    else {
        const size_t want = (hd.flags & 1u) ? buf.size() : (size_t)NP;
        if (std::fread(buf.data(), sizeof(float), want, f) != want) why = "truncated checkpoint";
        else if (std::fgetc(f) != EOF) why = "trailing bytes after the checkpoint";
    }
    std::fclose(f);
    if (!why.empty()) return nfail(PSC_ERR_IO, why + ": " + path);
    psc_net* n = nullptr;
    int st = psc_net_create(buf.data(), hip_stream, &n);
    if (st) return st;
    if (hd.flags & 1u) {
        if (hipMemcpy(n->m, buf.data() + NP, NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(n->v, buf.data() + 2 * NP, NP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            psc_net_free(n);
            return nfail(PSC_ERR_HIP, "optimiser state upload failed");
        }
        n->adam_t = hd.adam_t;
    }
    *out = n;
    return PSC_OK;
}

}  // extern "C"
