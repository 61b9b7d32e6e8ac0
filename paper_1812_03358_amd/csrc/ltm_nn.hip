// gfx950 kernels of the learned warm start: a 3-D convolutional
// encoder-decoder that maps A^T y to a starting volume for the solver.
//
// Activations are channels-last BF16 [D][H][W][C]; weights keep an FP32
// master copy [Cout][K] with K = tap * Cin + ci (tap = dz*9 + dy*3 + dx for
// 3x3x3, offsets -1..1, zero padding), packed to BF16 for the MFMA kernels.
//
// Convolution = implicit GEMM on v_mfma_f32_16x16x32_bf16 (FP32 accumulate):
// rows are output voxels, columns output channels, K runs over (tap, ci).
// Operand lane layout of the 16x16x32 instruction: lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7, and
// holds D[4 (l / 16) + i][l % 16], i = 0..3.
#include <algorithm>

#include "ltm_internal.h"
#include "ltm_nn.h"

namespace ltm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float((unsigned)v << 16); }

__device__ __forceinline__ u16 f2bf(float f)
{
    // round to nearest even (finite inputs); NaN stays NaN
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

union Frag {
    bf16x8 v;
    uint4 q;
    unsigned int w[4];
    u16 h[8];
};

// ---------------------------------------------------------------- conv forward
// One workgroup: 4 waves x MT tiles of 16 output voxels (flattened index),
// all NT x 16 output channels.  Input channels come from in0 (c0 channels)
// then in1 (c1 channels, the concatenated skip); the input grid is the
// output grid >> up (nearest upsampling fused into the read).
template <int KS, bool CIN1, int NT, int MT>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvFwd a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int V = a.D * a.H * a.W;
    const int Din = a.D >> a.up, Hin = a.H >> a.up, Win = a.W >> a.up;
    const int cin = a.c0 + a.c1;
    const int taps = KS * KS * KS;
    const int vbase = (blockIdx.x * 4 + wave) * (16 * MT);
    // this workgroup's output channels: tiles [blockIdx.y NT, blockIdx.y NT + NT)
    const int c16 = blockIdx.y * NT * 16;

    int vz[MT], vy[MT], vx[MT];
    bool vin[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int v = vbase + m * 16 + r;
        vin[m] = v < V;
        const int vv = vin[m] ? v : 0;
        vx[m] = vv % a.W;
        vy[m] = (vv / a.W) % a.H;
        vz[m] = vv / (a.W * a.H);
    }
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

    if (CIN1) {
        for (int k0 = 0; k0 < a.Kp; k0 += 32) {
            const int kk = k0 + 8 * kg;
            Frag A[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                A[m].q = uint4{0u, 0u, 0u, 0u};
                if (!vin[m]) continue;
                // one input channel: the 8 K values are 8 taps
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int tap = kk + j;
                    if (tap >= taps) continue;
                    const int dz = KS == 3 ? tap / 9 - 1 : 0, dy = KS == 3 ? (tap / 3) % 3 - 1 : 0,
                              dx = KS == 3 ? tap % 3 - 1 : 0;
                    const int z = vz[m] + dz, y = vy[m] + dy, x = vx[m] + dx;
                    if (z < 0 || z >= a.D || y < 0 || y >= a.H || x < 0 || x >= a.W) continue;
                    const size_t src = ((size_t)(z >> a.up) * Hin + (y >> a.up)) * Win + (x >> a.up);
                    A[m].h[j] = a.in0[src];
                }
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                Frag B;
                B.q = *reinterpret_cast<const uint4*>(a.wt + (size_t)(c16 + t * 16 + r) * a.Kp + kk);
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m].v, B.v, acc[m][t], 0, 0, 0);
            }
        }
    } else {
        // U K-steps at a time: all their operand loads are issued before
        // their MFMAs.  Loads are branch-free: an out-of-range tap or voxel
        // reads a valid address and selects zero; a K-step past Kp repeats
        // step k0 and is skipped.
        constexpr int U = 2;
        for (int k0 = 0; k0 < a.Kp; k0 += 32 * U) {
            Frag A[U][MT], B[U][NT];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int kk = (k0 + 32 * u < a.Kp ? k0 + 32 * u : k0) + 8 * kg;
                const int tap = kk / cin, ci = kk - tap * cin;
                const bool tapok = tap < taps;
                const int dz = KS == 3 ? tap / 9 - 1 : 0, dy = KS == 3 ? (tap / 3) % 3 - 1 : 0,
                          dx = KS == 3 ? tap % 3 - 1 : 0;
                // the 8 channels [ci, ci + 8) lie in one input (c0 % 8 == 0)
                const bool first = ci < a.c0;
                const u16* src_base = first ? a.in0 + ci : a.in1 + (ci - a.c0);
                const int cst = first ? a.c0 : a.c1;
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const int z = vz[m] + dz, y = vy[m] + dy, x = vx[m] + dx;
                    const bool ok = vin[m] && tapok && (unsigned)z < (unsigned)a.D &&
                                    (unsigned)y < (unsigned)a.H && (unsigned)x < (unsigned)a.W;
                    const size_t src =
                        ok ? ((size_t)(z >> a.up) * Hin + (y >> a.up)) * Win + (x >> a.up) : 0;
                    const uint4 q = *reinterpret_cast<const uint4*>(src_base + src * cst);
                    A[u][m].q = ok ? q : uint4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    B[u][t].q = *reinterpret_cast<const uint4*>(a.wt + (size_t)(c16 + t * 16 + r) * a.Kp + kk);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (k0 + 32 * u >= a.Kp) break;
#pragma unroll
                for (int t = 0; t < NT; ++t)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m][t] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[u][m].v, B[u][t].v, acc[m][t], 0, 0, 0);
            }
        }
    }
    // epilogue: bias, ReLU, store (BF16 or FP32, optionally split in two
    // channel ranges for the input gradient of a concatenation)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = c16 + t * 16 + r;
            if (co >= a.cout) continue;
            const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int v = vbase + m * 16 + 4 * kg + i;
                if (v >= V) continue;
                float val = acc[m][t][i] + b;
                if (a.relu) val = fmaxf(val, 0.0f);
                if (co < a.split) {
                    const size_t o = (size_t)v * a.split + co;
                    if (a.out_f32) reinterpret_cast<float*>(a.out)[o] = val;
                    else reinterpret_cast<u16*>(a.out)[o] = f2bf(val);
                } else {
                    const int c2 = a.cout - a.split;
                    const size_t o = (size_t)v * c2 + (co - a.split);
                    if (a.out_f32) reinterpret_cast<float*>(a.out2)[o] = val;
                    else reinterpret_cast<u16*>(a.out2)[o] = f2bf(val);
                }
            }
        }
}

// 3x3x3 convolution with at most 64 input channels, its input tile staged
// in LDS: a workgroup computes a 16 x 4 x TZ (x, y, z) block of output voxels
// (wave w: row y0 + w, its TZ tiles the TZ z planes, 16 voxels along x each)
// and stages the block's input halo (18 x 6 x (TZ + 2) voxels, all channels,
// zero outside the grid; the upsampled and the concatenated inputs resolved
// while staging) once, so each A fragment is one 16-byte LDS read instead of
// a global gather.  K runs over (tap, channel) as in the packed weights.
constexpr int kTX = 16, kTY = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2;

template <int NT, int TZ>
__global__ __launch_bounds__(256) void k_conv_fwd_lds(ConvFwd a)
{
    constexpr int kTZ = TZ, kHZ = TZ + 2;
    extern __shared__ uint4 hs4[];
    u16* hs = reinterpret_cast<u16*>(hs4);                 // [kHZ][kHY][kHX][cin]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int cin = a.c0 + a.c1;
    const int Din = a.D >> a.up, Hin = a.H >> a.up, Win = a.W >> a.up;
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    // stage the halo in 8-channel groups (16 bytes; c0 and c1 are multiples of 8)
    const int groups = cin >> 3;
    // groups is a power of two for 8, 16, 32 and 64 channels: split i by shifts
    const bool gpow2 = (groups & (groups - 1)) == 0;
    const int lg = __ffs(groups) - 1;
    for (int i = threadIdx.x; i < kHX * kHY * kHZ * groups; i += 256) {
        const int g = gpow2 ? (i & (groups - 1)) : i % groups;
        const int vox = gpow2 ? (i >> lg) : i / groups;
        const int hx = vox % kHX, hy = (vox / kHX) % kHY, hz = vox / (kHX * kHY);
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        const bool ok = (unsigned)x < (unsigned)a.W && (unsigned)y < (unsigned)a.H && (unsigned)z < (unsigned)a.D;
        const int xc = ok ? x : 0, yc = ok ? y : 0, zc = ok ? z : 0;
        const int ci = g * 8;
        const u16* src = ci < a.c0
            ? a.in0 + (((size_t)(zc >> a.up) * Hin + (yc >> a.up)) * Win + (xc >> a.up)) * a.c0 + ci
            : a.in1 + (((size_t)zc * a.H + yc) * a.W + xc) * a.c1 + (ci - a.c0);
        const uint4 q = *reinterpret_cast<const uint4*>(src);
        *reinterpret_cast<uint4*>(hs + (size_t)vox * cin + ci) = ok ? q : uint4{0u, 0u, 0u, 0u};
    }
    (void)Din;
    // per K-step and lane group: the halo offset (in u16) of the 8 channels
    // [ci, ci + 8) of tap (dz, dy, dx), relative to the lane's output voxel;
    // steps past the 27 taps (K padding, zero weights) point at offset 0 and
    // their A fragment is zeroed below
    const int nsteps = a.Kp >> 5;
    int* koff = reinterpret_cast<int*>(hs + (size_t)kHX * kHY * kHZ * cin);
    for (int i = threadIdx.x; i < nsteps * 4; i += 256) {
        const int k = (i >> 2) * 32 + 8 * (i & 3);
        const int tap = k / cin, ci = k - tap * cin;
        int off = 0;
        if (tap < 27) {
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            off = ((dz * kHY + dy) * kHX + dx) * cin + ci;
        }
        koff[i] = off;
    }
    __syncthreads();
    f32x4 acc[kTZ][NT];
#pragma unroll
    for (int m = 0; m < kTZ; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the lane's output voxel (x0 + r, y0 + wave, z0 + m) sits at halo
    // (1 + r, 1 + wave, 1 + m)
    const u16* abase = hs + (size_t)(((1 * kHY + 1 + wave) * kHX) + 1 + r) * cin;
    const size_t mstride = (size_t)kHY * kHX * cin;
    const u16* bbase = a.wt + (size_t)r * a.Kp + 8 * kg;
    if constexpr (NT == 1) {
        // two steps per trip with alternating operand buffers: the B fragments
        // and the offset of the next step are loaded while a step runs its MFMAs;
        // only the last step can hold K padding, so it alone (peeled) selects
        auto loadB = [&](Frag (&b)[NT], int ks) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                b[t].q = *reinterpret_cast<const uint4*>(bbase + (size_t)t * 16 * a.Kp + ks * 32);
        };
        auto mma = [&](const Frag (&b)[NT], int off, bool pad_step, int ks) {
            const bool ok = !pad_step || (ks * 32 + 8 * kg) < 27 * cin;
            Frag A[kTZ];
#pragma unroll
            for (int m = 0; m < kTZ; ++m) {
                A[m].q = *reinterpret_cast<const uint4*>(abase + m * mstride + off);
                if (pad_step) A[m].q = ok ? A[m].q : uint4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int m = 0; m < kTZ; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m].v, b[t].v, acc[m][t], 0, 0, 0);
        };
        Frag B0[NT], B1[NT];
        int off0 = koff[kg], off1 = 0;
        loadB(B0, 0);
        int ks = 0;
        for (; ks + 2 < nsteps; ks += 2) {
            loadB(B1, ks + 1);
            off1 = koff[(ks + 1) * 4 + kg];
            mma(B0, off0, false, ks);
            loadB(B0, ks + 2);
            off0 = koff[(ks + 2) * 4 + kg];
            mma(B1, off1, false, ks + 1);
        }
        if (ks + 1 < nsteps) {
            loadB(B1, ks + 1);
            off1 = koff[(ks + 1) * 4 + kg];
            mma(B0, off0, false, ks);
            mma(B1, off1, true, ks + 1);
        } else if (ks < nsteps) {
            mma(B0, off0, true, ks);
        }
    } else {
        // from 2 output tiles on: the weight fragments and halo offsets of the
        // next P steps are in flight while a step runs its NT x TZ MFMAs, and the
        // K-padding select runs on every step (one tile: two steps per trip with
        // alternating buffers and the padding step peeled, faster there --
        // measured 136 against 147-154 us for the 32-channel 128^3 layers)
        constexpr int P = NT == 2 ? 3 : 2;
        auto loadB = [&](Frag (&b)[NT], int ks) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                b[t].q = *reinterpret_cast<const uint4*>(bbase + (size_t)t * 16 * a.Kp + ks * 32);
        };
        auto mma = [&](const Frag (&b)[NT], int off, int ks) {
            const bool ok = ks < nsteps - 1 || (ks * 32 + 8 * kg) < 27 * cin;
            Frag A[kTZ];
#pragma unroll
            for (int m = 0; m < kTZ; ++m) {
                A[m].q = *reinterpret_cast<const uint4*>(abase + m * mstride + off);
                A[m].q = ok ? A[m].q : uint4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int m = 0; m < kTZ; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[m].v, b[t].v, acc[m][t], 0, 0, 0);
        };
        Frag Bq[P][NT];
        int offq[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            offq[p] = p < nsteps ? koff[p * 4 + kg] : 0;
            if (p < nsteps) loadB(Bq[p], p);
        }
        for (int ks0 = 0; ks0 < nsteps; ks0 += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int ks = ks0 + p;
                if (ks < nsteps) {
                    mma(Bq[p], offq[p], ks);
                    if (ks + P < nsteps) {
                        loadB(Bq[p], ks + P);
                        offq[p] = koff[(ks + P) * 4 + kg];
                    }
                }
            }
        }
    }
    // epilogue: output row 4 kg + i of tile m is voxel (x0 + 4 kg + i, y0 + wave, z0 + m)
    const int y = y0 + wave;
#pragma unroll
    for (int m = 0; m < kTZ; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = t * 16 + r;
            if (co >= a.cout) continue;
            const int z = z0 + m;
            if (z >= a.D || y >= a.H) continue;
            const float b = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = x0 + 4 * kg + i;
                if (x >= a.W) continue;
                const size_t v = ((size_t)z * a.H + y) * a.W + x;
                float val = acc[m][t][i] + b;
                if (a.relu) val = fmaxf(val, 0.0f);
                if (co < a.split) {
                    const size_t o = v * a.split + co;
                    if (a.out_f32) reinterpret_cast<float*>(a.out)[o] = val;
                    else reinterpret_cast<u16*>(a.out)[o] = f2bf(val);
                } else {
                    const int c2 = a.cout - a.split;
                    const size_t o = v * c2 + (co - a.split);
                    if (a.out_f32) reinterpret_cast<float*>(a.out2)[o] = val;
                    else reinterpret_cast<u16*>(a.out2)[o] = f2bf(val);
                }
            }
        }
}

// 3x3x3 convolution of a single input channel (the network's input layer),
// up to 16 output channels: 27 MACs per output channel, so FP32 FMAs on the
// BF16 values (their products are exact in FP32) instead of MFMAs whose K
// values would each be a separately gathered tap.  A workgroup stages the
// 18 x 6 x 6 input halo of a 16 x 4 x 4 output block in LDS; each thread
// computes one output voxel's channels.  The weights are the same for every
// lane (read with uniform addresses, so they arrive through scalar loads).
__global__ __launch_bounds__(256) void k_conv_fwd_c1(ConvFwd a)
{
    __shared__ float halo[6][6][18];
    const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 4, z0 = blockIdx.z * 4;
    const int Hin = a.H >> a.up, Win = a.W >> a.up;
    for (int i = threadIdx.x; i < 18 * 6 * 6; i += 256) {
        const int hx = i % 18, hy = (i / 18) % 6, hz = i / 108;
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        const bool ok = (unsigned)x < (unsigned)a.W && (unsigned)y < (unsigned)a.H && (unsigned)z < (unsigned)a.D;
        halo[hz][hy][hx] =
            ok ? bf2f(a.in0[((size_t)(z >> a.up) * Hin + (y >> a.up)) * Win + (x >> a.up)]) : 0.0f;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = (threadIdx.x >> 4) & 3, tz = threadIdx.x >> 6;
    const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
    if (x >= a.W || y >= a.H || z >= a.D) return;
    float v[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) v[t] = halo[tz + t / 9][ty + (t / 3) % 3][tx + t % 3];
    const size_t vox = ((size_t)z * a.H + y) * a.W + x;
    float out[16];
#pragma unroll
    for (int co = 0; co < 16; ++co) {
        if (co >= a.cout) {
            out[co] = 0.0f;
            continue;
        }
        const u16* wr = a.wt + (size_t)co * a.Kp;
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 27; ++t) acc = fmaf(bf2f(wr[t]), v[t], acc);
        acc += a.bias ? a.bias[co] : 0.0f;
        out[co] = a.relu ? fmaxf(acc, 0.0f) : acc;
    }
    if (!a.out_f32 && a.split == 16 && a.cout == 16) {
        // one voxel's 16 BF16 channels: two 16-byte stores
        Frag lo, hi;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            lo.h[j] = f2bf(out[j]);
            hi.h[j] = f2bf(out[8 + j]);
        }
        uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<u16*>(a.out) + vox * 16);
        dst[0] = lo.q;
        dst[1] = hi.q;
        return;
    }
    for (int co = 0; co < 16; ++co) {
        if (co >= a.cout) break;
        if (co < a.split) {
            const size_t o = vox * a.split + co;
            if (a.out_f32) reinterpret_cast<float*>(a.out)[o] = out[co];
            else reinterpret_cast<u16*>(a.out)[o] = f2bf(out[co]);
        } else {
            const size_t o = vox * (a.cout - a.split) + (co - a.split);
            if (a.out_f32) reinterpret_cast<float*>(a.out2)[o] = out[co];
            else reinterpret_cast<u16*>(a.out2)[o] = f2bf(out[co]);
        }
    }
}

// ---------------------------------------------------------------- wgrad
// dW[co][k] += sum_v dY[v][co] X_k[v], k = tap * Cin + ci, X_k the input
// shifted by the tap (and upsampled when up = 1).  MFMA rows are output
// channels, columns are k, the reduction runs over 32 voxels of one output
// z-slice at a time.  A workgroup's 4 waves own 4 (co, k) tiles of one share
// of one slice (gridDim.z shares of its 32-voxel groups) and add them into
// the FP32 gradient with atomics.
template <int KS>
__global__ __launch_bounds__(256) void k_conv_wgrad(ConvWgrad a)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int n_co = (a.cout + 15) / 16;
    const int n_k = (a.K + 15) / 16;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= n_co * n_k) return;
    const int cot = tile % n_co, kt = tile / n_co;
    const int z = blockIdx.y;
    const int HW = a.H * a.W;
    const int Hin = a.H >> a.up, Win = a.W >> a.up;
    const int cin = a.c0 + a.c1;
    const int co = cot * 16 + r;           // A row of this lane
    const int k = kt * 16 + r;             // B column of this lane
    const bool kvalid = k < a.K;
    const int tap = kvalid ? k / cin : 0, ci = kvalid ? k - tap * cin : 0;
    const int dz = KS == 3 ? tap / 9 - 1 : 0, dy = KS == 3 ? (tap / 3) % 3 - 1 : 0,
              dx = KS == 3 ? tap % 3 - 1 : 0;
    const int zz = z + dz;
    const bool zin = kvalid && zz >= 0 && zz < a.D;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // this workgroup's share of the slice (gridDim.z shares of 32-voxel groups)
    const int ngroups = (HW + 31) / 32;
    const int g0 = (int)(((long long)ngroups * blockIdx.z) / gridDim.z);
    const int g1 = (int)(((long long)ngroups * (blockIdx.z + 1)) / gridDim.z);
    for (int v0 = g0 * 32; v0 < g1 * 32; v0 += 32) {
        Frag A, B;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int v = v0 + 8 * kg + j;
            u16 av = 0, bv = 0;
            if (v < HW) {
                if (co < a.cout) av = a.dy[((size_t)z * HW + v) * a.cout + co];
                const int y = v / a.W + dy, x = v % a.W + dx;
                if (zin && y >= 0 && y < a.H && x >= 0 && x < a.W) {
                    const size_t src = ((size_t)(zz >> a.up) * Hin + (y >> a.up)) * Win + (x >> a.up);
                    bv = ci < a.c0 ? a.in0[src * a.c0 + ci] : a.in1[src * a.c1 + (ci - a.c0)];
                }
            }
            A.h[j] = av;
            B.h[j] = bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.v, B.v, acc, 0, 0, 0);
    }
    // D[row = 4 kg + i][col = r]: row is the output channel, col is k
    const int kc = kt * 16 + r;
    if (kc >= a.K) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = cot * 16 + 4 * kg + i;
        if (c < a.cout && acc[i] != 0.0f) unsafeAtomicAdd(&a.dw[(size_t)c * a.K + kc], acc[i]);
    }
}

// k_conv_wgrad for grids whose H and W are powers of two (H W a multiple of
// 32) and cout a multiple of 16: voxel coordinates by shifts, no branches in
// the operand loads (an out-of-range tap reads a valid address and selects
// zero), the input base pointer and channel stride of each lane hoisted, and
// each wave owning NK k-tiles of one output-channel tile, so one dY fragment
// feeds NK MFMAs.
template <int KS, int NK>
__global__ __launch_bounds__(256) void k_conv_wgrad_pow2(ConvWgrad a, int lw, int lh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int n_co = a.cout >> 4;
    const int n_kg = ((a.K + 15) / 16 + NK - 1) / NK;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= n_co * n_kg) return;
    const int cot = tile % n_co, kgi = tile / n_co;
    const int z = blockIdx.y;
    const int W = 1 << lw, H = 1 << lh, HW = W * H;
    const int Hin = H >> a.up, Win = W >> a.up;
    const int cin = a.c0 + a.c1;
    const u16* dyz = a.dy + (size_t)z * HW * a.cout + cot * 16 + r;
    // per k-tile: this lane's B column k = tap * cin + ci
    const u16* base[NK];
    int cst[NK], ddy[NK], ddx[NK], zoff[NK];
    bool live[NK];
#pragma unroll
    for (int t = 0; t < NK; ++t) {
        const int k = (kgi * NK + t) * 16 + r;
        const bool kv = k < a.K;
        const int tap = kv ? k / cin : 0, ci = kv ? k - tap * cin : 0;
        const int dz = KS == 3 ? tap / 9 - 1 : 0;
        ddy[t] = KS == 3 ? (tap / 3) % 3 - 1 : 0;
        ddx[t] = KS == 3 ? tap % 3 - 1 : 0;
        const int zz = z + dz;
        live[t] = kv && zz >= 0 && zz < a.D;
        zoff[t] = live[t] ? (zz >> a.up) * Hin * Win : 0;
        base[t] = ci < a.c0 ? a.in0 + ci : a.in1 + (ci - a.c0);
        cst[t] = ci < a.c0 ? a.c0 : a.c1;
    }
    f32x4 acc[NK];
#pragma unroll
    for (int t = 0; t < NK; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // a wave walks a whole slice, U voxel groups at a time: all their loads
    // are issued before their MFMAs (a group past the slice loads group 0
    // and is skipped)
    constexpr int U = 4;
    // this workgroup's share of the slice's voxel groups (gridDim.z shares)
    const int ngroups = HW >> 5;
    const int sb = (int)(((long long)ngroups * blockIdx.z) / gridDim.z);
    const int nsteps = (int)(((long long)ngroups * (blockIdx.z + 1)) / gridDim.z);
    for (int s0 = sb; s0 < nsteps; s0 += U) {
        Frag A[U], B[U][NK];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int vb = (s0 + u < nsteps ? s0 + u : sb) * 32 + 8 * kg;
#pragma unroll
            for (int j = 0; j < 8; ++j) A[u].h[j] = dyz[(size_t)(vb + j) * a.cout];
            const int y0 = vb >> lw, x0 = vb & (W - 1);   // the 8 voxels share a row (W >= 8)
#pragma unroll
            for (int t = 0; t < NK; ++t) {
                const int y = y0 + ddy[t];
                const bool rowok = live[t] && (unsigned)y < (unsigned)H;
                const int rowoff = zoff[t] + (rowok ? (y >> a.up) : 0) * Win;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int x = x0 + j + ddx[t];
                    const bool ok = rowok && (unsigned)x < (unsigned)W;
                    const u16 val = base[t][(size_t)(rowoff + (ok ? (x >> a.up) : 0)) * cst[t]];
                    B[u][t].h[j] = ok ? val : (u16)0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (s0 + u >= nsteps) break;
#pragma unroll
            for (int t = 0; t < NK; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[u].v, B[u][t].v, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) {
        const int kc = (kgi * NK + t) * 16 + r;
        if (kc >= a.K) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = cot * 16 + 4 * kg + i;
            if (acc[t][i] != 0.0f) unsafeAtomicAdd(&a.dw[(size_t)c * a.K + kc], acc[t][i]);
        }
    }
}

// Weight gradient of a 3x3x3 convolution for rows whose width is a multiple
// of XC (32, 64 or 128) voxels and Cin, Cout multiples of 16.  A tap's x shift
// is moved from the input onto dY: sum_x dY[x] X[x + dx] = sum_x' dY[x' - dx]
// X[x'], each input position x' paired by the unit that holds it.  A unit is
// XC voxels (chunk) of one output row (z, y).  Per unit a workgroup holds in
// LDS the 9 input rows (z + dz, y + dy) the taps reach, at the unit's own x
// range and for one 16-channel input tile, and the unit's dY for one
// 16-channel output tile in three copies shifted by dx = -1, 0, 1 (zeros
// outside the grid; upsampling and concatenation resolved while staging).
// Both are stored transposed, [channel][x], so every MFMA operand (8
// consecutive voxels of one channel) is one aligned 16-byte LDS read, and one
// input fragment feeds the three taps that differ only in dx.  Units run over
// (z, chunk, y) with y fastest: the input rows sit in a ring of 3 x 3 slots
// (slot (dz, y' mod 3)), so a unit after its y - 1 neighbour loads only the 3
// rows y + 1; and the next unit's loads are issued into registers before the
// current unit's MFMAs.  A workgroup owns (output tile, input tile, a
// contiguous share of the units); wave w holds the 9 k-tiles of dy = w - 1 in
// registers over its share and adds them into dw once.
template <int XC>
struct WgradStage {
    static constexpr int NX8 = XC / 8;
    static constexpr int NIT = (9 * 2 * NX8 + 191) / 192;     // input items per thread (a full stage)
    static constexpr int NDI = (2 * (XC + 2) + 191) / 192;    // dY items per thread
    Frag q[NIT][8];
    Frag f[NDI];
};

template <int XC>
__device__ __forceinline__ void wgrad_load(const ConvWgrad& a, int cit, int cot, int z, int y, int x0, bool full,
                                           WgradStage<XC>& st)
{
    constexpr int NX8 = XC / 8;
    const int nitems = (full ? 9 : 3) * 2 * NX8;
    const int Hin = a.H >> a.up, Win = a.W >> a.up;
#pragma unroll
    for (int it = 0; it < WgradStage<XC>::NIT; ++it) {
        const int i = (int)threadIdx.x + 192 * it;
        const int x8 = i % NX8, g = (i / NX8) & 1, rs = i / (2 * NX8);
        const int dzi = full ? rs / 3 : rs, k = full ? rs % 3 : 2;
        const int zz = z + dzi - 1, yy = y + k - 1;
        const int ci = cit * 16 + g * 8;
        const int xb = x0 + x8 * 8;
        if (i < nitems && (unsigned)zz < (unsigned)a.D && (unsigned)yy < (unsigned)a.H) {
            if (ci < a.c0) {
                const u16* src = a.in0 + ((size_t)(zz >> a.up) * Hin + (yy >> a.up)) * Win * a.c0 + ci;
#pragma unroll
                for (int jx = 0; jx < 8; ++jx)
                    st.q[it][jx].q = *reinterpret_cast<const uint4*>(src + (size_t)((xb + jx) >> a.up) * a.c0);
            } else {
                const u16* src = a.in1 + ((size_t)zz * a.H + yy) * a.W * a.c1 + (ci - a.c0);
#pragma unroll
                for (int jx = 0; jx < 8; ++jx)
                    st.q[it][jx].q = *reinterpret_cast<const uint4*>(src + (size_t)(xb + jx) * a.c1);
            }
        } else {
#pragma unroll
            for (int jx = 0; jx < 8; ++jx) st.q[it][jx].q = uint4{0u, 0u, 0u, 0u};
        }
    }
    const size_t rowbase = ((size_t)z * a.H + y) * a.W;
#pragma unroll
    for (int it = 0; it < WgradStage<XC>::NDI; ++it) {
        const int i = (int)threadIdx.x + 192 * it;
        const int h = i >> 1, half = i & 1;
        const int x = x0 - 1 + h;
        st.f[it].q = (i < 2 * (XC + 2) && (unsigned)x < (unsigned)a.W)
            ? *reinterpret_cast<const uint4*>(a.dy + (rowbase + x) * a.cout + cot * 16 + half * 8)
            : uint4{0u, 0u, 0u, 0u};
    }
}

template <int XC>
__device__ __forceinline__ void wgrad_store(int y, bool full, const WgradStage<XC>& st, u16* xs, u16* dys)
{
    constexpr int NX8 = XC / 8, XS = XC + 8;
    const int nitems = (full ? 9 : 3) * 2 * NX8;
#pragma unroll
    for (int it = 0; it < WgradStage<XC>::NIT; ++it) {
        const int i = (int)threadIdx.x + 192 * it;
        if (i >= nitems) continue;
        const int x8 = i % NX8, g = (i / NX8) & 1, rs = i / (2 * NX8);
        const int dzi = full ? rs / 3 : rs, k = full ? rs % 3 : 2;
        const int slot = dzi * 3 + (y + k + 2) % 3;               // input row y + k - 1 -> slot (dz, y' mod 3)
        u16* dst = xs + (slot * 16 + g * 8) * XS + x8 * 8;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // channel j of voxels 2m, 2m + 1 -> one dword (low, high half)
            const unsigned sel = (j & 1) ? 0x07060302u : 0x05040100u;
            uint4 o;
            o.x = __builtin_amdgcn_perm(st.q[it][1].w[j >> 1], st.q[it][0].w[j >> 1], sel);
            o.y = __builtin_amdgcn_perm(st.q[it][3].w[j >> 1], st.q[it][2].w[j >> 1], sel);
            o.z = __builtin_amdgcn_perm(st.q[it][5].w[j >> 1], st.q[it][4].w[j >> 1], sel);
            o.w = __builtin_amdgcn_perm(st.q[it][7].w[j >> 1], st.q[it][6].w[j >> 1], sel);
            *reinterpret_cast<uint4*>(dst + j * XS) = o;
        }
    }
    // dY halo x0 - 1 + h: copy d (dx = d - 1) holds dY[x0 + i - dx] at i = h + d - 2
#pragma unroll
    for (int it = 0; it < WgradStage<XC>::NDI; ++it) {
        const int i = (int)threadIdx.x + 192 * it;
        if (i >= 2 * (XC + 2)) continue;
        const int h = i >> 1, half = i & 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int ix = h + d - 2;
            if ((unsigned)ix < (unsigned)XC) {
#pragma unroll
                for (int j = 0; j < 8; ++j) dys[(d * 16 + half * 8 + j) * XS + ix] = st.f[it].h[j];
            }
        }
    }
}

template <int XC>
__global__ __launch_bounds__(192) void k_conv_wgrad_rows(ConvWgrad a, int nshare)
{
    constexpr int XS = XC + 8;                   // LDS row stride (elements), padded against bank conflicts
    extern __shared__ uint4 sm4[];
    u16* xs = reinterpret_cast<u16*>(sm4);       // [9 slots][16 channels][XS]
    u16* dys = xs + 9 * 16 * XS;                 // [3 shifts][16 channels][XS]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int n_co = a.cout >> 4;
    const int cot = blockIdx.x % n_co, cit = blockIdx.x / n_co;
    const int cin = a.c0 + a.c1;
    const int chunks = a.W / XC;
    const int nunits = a.D * chunks * a.H;
    const int u0 = (int)(((long long)nunits * blockIdx.y) / nshare);
    const int u1 = (int)(((long long)nunits * (blockIdx.y + 1)) / nshare);
    f32x4 acc[3][3];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[s][d] = f32x4{0.f, 0.f, 0.f, 0.f};
    // unit -> (z, chunk, y), y fastest
    auto coords = [&](int unit, int& z, int& y, int& x0) {
        const int zc = unit / a.H;
        y = unit - zc * a.H;
        z = zc / chunks;
        x0 = (zc - z * chunks) * XC;
    };
    WgradStage<XC> st;
    int z, y, x0;
    if (u0 < u1) {
        coords(u0, z, y, x0);
        wgrad_load<XC>(a, cit, cot, z, y, x0, true, st);
    }
    for (int unit = u0; unit < u1; ++unit) {
        const bool full = unit == u0 || y == 0;
        const int ycur = y;
        __syncthreads();   // the previous unit's fragments are read
        wgrad_store<XC>(ycur, full, st, xs, dys);
        __syncthreads();
        if (unit + 1 < u1) {
            coords(unit + 1, z, y, x0);
            wgrad_load<XC>(a, cit, cot, z, y, x0, y == 0, st);
        }
        // wave w: dy = w - 1, input row y' = ycur + w - 1 in slot (s, y' mod 3)
        const int ks = (ycur + wave + 2) % 3;
#pragma unroll
        for (int gv = 0; gv < XC; gv += 32) {
            Frag A[3];
#pragma unroll
            for (int d = 0; d < 3; ++d)
                A[d].q = *reinterpret_cast<const uint4*>(dys + (d * 16 + r) * XS + gv + 8 * kg);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                Frag B;
                B.q = *reinterpret_cast<const uint4*>(xs + ((s * 3 + ks) * 16 + r) * XS + gv + 8 * kg);
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    acc[s][d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[d].v, B.v, acc[s][d], 0, 0, 0);
            }
        }
    }
    // D[4 kg + i][r]: output channel cot 16 + 4 kg + i, input channel
    // cit 16 + r of tap (dz = s - 1, dy = wave - 1, dx = d - 1)
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int k = ((s * 3 + wave) * 3 + d) * cin + cit * 16 + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = cot * 16 + 4 * kg + i;
                if (acc[s][d][i] != 0.0f) unsafeAtomicAdd(&a.dw[(size_t)c * a.K + k], acc[s][d][i]);
            }
        }
}

template <int XC>
hipError_t wgrad_rows(const ConvWgrad& a, hipStream_t s)
{
    const int tiles = (a.cout / 16) * ((a.c0 + a.c1) / 16);
    const int units = a.D * a.H * (a.W / XC);
    // shares of the units per (output tile, input tile) until ~512 workgroups
    // run (two per CU); each share adds its partial sums into dw
    const int shares = std::max(1, std::min(units, 512 / tiles));
    const size_t lds = (size_t)12 * 16 * (XC + 8) * sizeof(u16);
    hipLaunchKernelGGL((k_conv_wgrad_rows<XC>), dim3(tiles, shares), dim3(192), lds, s, a, shares);
    return hipGetLastError();
}

// Weight gradient of a 3x3x3 convolution with one input channel (the input
// layer) on rows of XC (32, 64 or 128) voxels.  With one channel, the 9 input
// rows (z + dz, y + dy) a unit's taps reach are the columns of one MFMA B
// operand (9 of 16 used), staged in three copies shifted by dx = -1, 0, 1
// (zeros outside the grid); the unit's dY of one 16-channel output tile is
// staged transposed, [co][x].  Each 32 voxels take 3 MFMAs (one per x shift)
// into D[co][row], tap = row * 3 + d; a wave takes every fourth group of 32
// voxels, and the workgroup sums its waves in LDS and adds into dw once.
template <int XC>
__global__ __launch_bounds__(256) void k_conv_wgrad_c1(ConvWgrad a, int nshare)
{
    constexpr int XS = XC + 8;
    __shared__ __align__(16) u16 xs[3 * 16 * XS];   // [shift][row][x]; rows 9..15 stay zero
    __shared__ __align__(16) u16 dys[16 * XS];      // [co][x]
    __shared__ float red[27 * 16];                  // [tap][co]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, kg = lane >> 4;
    const int cot = blockIdx.x;
    const int chunks = a.W / XC;
    const int nunits = a.D * a.H * chunks;
    const int u0 = (int)(((long long)nunits * blockIdx.y) / nshare);
    const int u1 = (int)(((long long)nunits * (blockIdx.y + 1)) / nshare);
    for (int i = threadIdx.x; i < 3 * 16 * XS; i += 256) xs[i] = 0;
    for (int i = threadIdx.x; i < 27 * 16; i += 256) red[i] = 0.0f;
    f32x4 acc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int unit = u0; unit < u1; ++unit) {
        const int row = unit / chunks, x0 = (unit - row * chunks) * XC;
        const int z = row / a.H, y = row - z * a.H;
        __syncthreads();   // the previous unit's fragments are read (and the clears done)
        // input halo x0 - 1 + h: copy d (dx = d - 1) holds X[x0 + i + dx] at i = h - d
        for (int i = threadIdx.x; i < 9 * (XC + 2); i += 256) {
            const int rr = i / (XC + 2), h = i - rr * (XC + 2);
            const int zz = z + rr / 3 - 1, yy = y + rr % 3 - 1, x = x0 - 1 + h;
            u16 v = 0;
            if ((unsigned)zz < (unsigned)a.D && (unsigned)yy < (unsigned)a.H && (unsigned)x < (unsigned)a.W)
                v = a.in0[((size_t)zz * a.H + yy) * a.W + x];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int ix = h - d;
                if ((unsigned)ix < (unsigned)XC) xs[(d * 16 + rr) * XS + ix] = v;
            }
        }
        for (int i = threadIdx.x; i < XC * 2; i += 256) {
            const int x = i >> 1, half = i & 1;
            Frag f;
            f.q = *reinterpret_cast<const uint4*>(a.dy + ((size_t)row * a.W + x0 + x) * a.cout + cot * 16 + half * 8);
#pragma unroll
            for (int j = 0; j < 8; ++j) dys[(half * 8 + j) * XS + x] = f.h[j];
        }
        __syncthreads();
        for (int gv = wave * 32; gv < XC; gv += 128) {
            Frag A;
            A.q = *reinterpret_cast<const uint4*>(dys + r * XS + gv + 8 * kg);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Frag B;
                B.q = *reinterpret_cast<const uint4*>(xs + (d * 16 + r) * XS + gv + 8 * kg);
                acc[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.v, B.v, acc[d], 0, 0, 0);
            }
        }
    }
    // D[4 kg + i][r]: output channel cot 16 + 4 kg + i, input row r (< 9),
    // x shift d -> tap r * 3 + d
    if (r < 9) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (acc[d][i] != 0.0f) atomicAdd(&red[(r * 3 + d) * 16 + 4 * kg + i], acc[d][i]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 27 * 16; i += 256) {
        const int tap = i >> 4, co = i & 15;
        if (red[i] != 0.0f) unsafeAtomicAdd(&a.dw[(size_t)(cot * 16 + co) * a.K + tap], red[i]);
    }
}

template <int XC>
hipError_t wgrad_c1(const ConvWgrad& a, hipStream_t s)
{
    const int cot = a.cout / 16;
    const int units = a.D * a.H * (a.W / XC);
    // shares of the units until ~1024 workgroups run; each adds 16 x 27 sums
    const int shares = std::max(1, std::min(units, 1024 / cot));
    hipLaunchKernelGGL((k_conv_wgrad_c1<XC>), dim3(cot, shares), dim3(256), 0, s, a, shares);
    return hipGetLastError();
}

// Weight gradient of a 1x1x1 convolution to one output channel (the output
// layer): dw[ci] += sum_v dY[v] X[v][ci].  Each thread sums its voxels' CIN
// channels in registers (16-byte loads), then waves and the workgroup combine
// them, one atomic per channel and workgroup.
template <int CIN>
__global__ __launch_bounds__(256) void k_wgrad_1x1_out1(ConvWgrad a, size_t nvox)
{
    __shared__ float red[CIN];
    if (threadIdx.x < CIN) red[threadIdx.x] = 0.0f;
    __syncthreads();
    float sum[CIN];
#pragma unroll
    for (int c = 0; c < CIN; ++c) sum[c] = 0.0f;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (size_t)gridDim.x * 256) {
        const float g = bf2f(a.dy[v]);
        const u16* x = a.in0 + v * CIN;
#pragma unroll
        for (int c8 = 0; c8 < CIN; c8 += 8) {
            Frag q;
            q.q = *reinterpret_cast<const uint4*>(x + c8);
#pragma unroll
            for (int j = 0; j < 8; ++j) sum[c8 + j] = fmaf(g, bf2f(q.h[j]), sum[c8 + j]);
        }
    }
#pragma unroll
    for (int c = 0; c < CIN; ++c) {
        float t = sum[c];
        for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
        if ((threadIdx.x & 63) == 0 && t != 0.0f) atomicAdd(&red[c], t);
    }
    __syncthreads();
    if (threadIdx.x < CIN && red[threadIdx.x] != 0.0f) unsafeAtomicAdd(&a.dw[threadIdx.x], red[threadIdx.x]);
}

// 1x1x1 convolution to one output channel (the output layer): each voxel's
// CIN channels (16-byte loads) dotted with the weight row, plus bias, ReLU if
// asked.
template <int CIN>
__global__ __launch_bounds__(256) void k_conv1x1_out1(ConvFwd a, size_t nvox)
{
    float w[CIN];
#pragma unroll
    for (int c8 = 0; c8 < CIN; c8 += 8) {
        Frag q;
        q.q = *reinterpret_cast<const uint4*>(a.wt + c8);
#pragma unroll
        for (int j = 0; j < 8; ++j) w[c8 + j] = bf2f(q.h[j]);
    }
    const float b = a.bias ? a.bias[0] : 0.0f;
    for (size_t v = (size_t)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (size_t)gridDim.x * 256) {
        const u16* x = a.in0 + v * CIN;
        float acc = 0.0f;
#pragma unroll
        for (int c8 = 0; c8 < CIN; c8 += 8) {
            Frag q;
            q.q = *reinterpret_cast<const uint4*>(x + c8);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc = fmaf(bf2f(q.h[j]), w[c8 + j], acc);
        }
        acc += b;
        if (a.relu) acc = fmaxf(acc, 0.0f);
        if (a.out_f32) reinterpret_cast<float*>(a.out)[v] = acc;
        else reinterpret_cast<u16*>(a.out)[v] = f2bf(acc);
    }
}

// ---------------------------------------------------------------- elementwise
// Pack FP32 master weights [Cout][K] into the BF16 forward layout
// [NT*16][Kp] and the input-gradient layout [Cin_pad][Kp'] (flipped taps,
// in/out channels swapped), zero padded.
__global__ void k_pack(const float* __restrict__ w, int cout, int cin, int taps, u16* __restrict__ wf,
                       int rows_f, int kp_f, u16* __restrict__ wb, int rows_b, int kp_b)
{
    const int K = taps * cin;
    const size_t nf = (size_t)rows_f * kp_f, nb = wb ? (size_t)rows_b * kp_b : 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf + nb;
         i += (size_t)gridDim.x * blockDim.x) {
        if (i < nf) {
            const int row = (int)(i / kp_f), k = (int)(i % kp_f);
            wf[i] = (row < cout && k < K) ? f2bf(w[(size_t)row * K + k]) : (u16)0;
        } else {
            const size_t j = i - nf;
            const int c = (int)(j / kp_b), kb = (int)(j % kp_b);   // c: input channel
            u16 v = 0;
            if (c < cin && kb < taps * cout) {
                const int tb = kb / cout, o = kb - tb * cout;
                const int t = taps - 1 - tb;                        // flipped tap
                v = f2bf(w[(size_t)o * K + t * cin + c]);
            }
            wb[j] = v;
        }
    }
}

// y = 2x2x2 max of x (BF16, channels-last), arg = winning child 0..7.
__global__ void k_maxpool(const u16* __restrict__ x, u16* __restrict__ y, unsigned char* __restrict__ arg,
                          int D, int H, int W, int C)
{
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const size_t n = (size_t)Do * Ho * Wo * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int xo = (int)(v % Wo), yo = (int)((v / Wo) % Ho), zo = (int)(v / ((size_t)Wo * Ho));
        float best = -INFINITY;
        int bi = 0;
        for (int q = 0; q < 8; ++q) {
            const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
            const float val = bf2f(x[(((size_t)z * H + yy) * W + xx) * C + c]);
            if (val > best) {
                best = val;
                bi = q;
            }
        }
        y[i] = f2bf(best);
        arg[i] = (unsigned char)bi;
    }
}

// dx[child] += dy at the winning child (FP32 accumulate into dx).
__global__ void k_maxpool_bwd(const float* __restrict__ dy, const unsigned char* __restrict__ arg,
                              float* __restrict__ dx, int D, int H, int W, int C)
{
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const size_t n = (size_t)Do * Ho * Wo * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int xo = (int)(v % Wo), yo = (int)((v / Wo) % Ho), zo = (int)(v / ((size_t)Wo * Ho));
        const int q = arg[i];
        const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
        dx[(((size_t)z * H + yy) * W + xx) * C + c] += dy[i];
    }
}

// dlow = sum of the 8 children of dhigh (backward of nearest 2x upsampling).
__global__ void k_sumpool(const float* __restrict__ dh, float* __restrict__ dl, int D, int H, int W, int C,
                          int accumulate)
{
    const int Do = D / 2, Ho = H / 2, Wo = W / 2;
    const size_t n = (size_t)Do * Ho * Wo * C;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const size_t v = i / C;
        const int xo = (int)(v % Wo), yo = (int)((v / Wo) % Ho), zo = (int)(v / ((size_t)Wo * Ho));
        float s = 0.0f;
        for (int q = 0; q < 8; ++q) {
            const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
            s += dh[(((size_t)z * H + yy) * W + xx) * C + c];
        }
        dl[i] = accumulate ? dl[i] + s : s;
    }
}

// g = dOut * (out > 0) as BF16 (the MFMA operand) and its per-channel sum.
// When C divides the grid stride (C a power of two up to 256) every thread
// keeps one channel: its sum stays in a register, lanes of one channel are
// combined with wave shuffles and each wave adds C values into LDS.
__global__ void k_relu_mask_pc(const float* __restrict__ dout, const u16* __restrict__ out, int relu,
                               u16* __restrict__ g, float* __restrict__ dbias, size_t n, int C)
{
    extern __shared__ float sb[];
    for (int c = threadIdx.x; c < C; c += blockDim.x) sb[c] = 0.0f;
    __syncthreads();
    float part = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = dout[i];
        if (relu && !(bf2f(out[i]) > 0.0f)) v = 0.0f;
        const u16 b = f2bf(v);
        g[i] = b;
        part += bf2f(b);
    }
    // lanes l and l + C (C < 64) hold the same channel
    for (int o = 32; o >= C && o > 0; o >>= 1) part += __shfl_xor(part, o);
    const int lane = threadIdx.x & 63;
    if (lane < C && part != 0.0f) atomicAdd(&sb[threadIdx.x % C], part);
    __syncthreads();
    if (dbias)
        for (int c = threadIdx.x; c < C; c += blockDim.x)
            if (sb[c] != 0.0f) unsafeAtomicAdd(&dbias[c], sb[c]);
}

// k_relu_mask_pc over 8 consecutive elements per thread and step (16-byte
// loads and stores).  C divides 2048, so a thread's 8 elements keep their
// channels (8 t + j) mod C through the grid-stride loop: the 8 sums stay in
// registers, lanes holding the same channels are combined with wave
// shuffles, and the rest reach LDS once per wave.
__global__ __launch_bounds__(256) void k_relu_mask_v8(const float* __restrict__ dout, const u16* __restrict__ out,
                                                      int relu, u16* __restrict__ g, float* __restrict__ dbias,
                                                      size_t n8, int C)
{
    extern __shared__ float sb[];
    for (int c = threadIdx.x; c < C; c += blockDim.x) sb[c] = 0.0f;
    __syncthreads();
    float part[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < n8; i += (size_t)gridDim.x * blockDim.x) {
        const float4 d0 = reinterpret_cast<const float4*>(dout)[2 * i];
        const float4 d1 = reinterpret_cast<const float4*>(dout)[2 * i + 1];
        float v[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        if (relu) {
            Frag o;
            o.q = reinterpret_cast<const uint4*>(out)[i];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (!(bf2f(o.h[j]) > 0.0f)) v[j] = 0.0f;
        }
        Frag b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            b.h[j] = f2bf(v[j]);
            part[j] += bf2f(b.h[j]);
        }
        reinterpret_cast<uint4*>(g)[i] = b.q;
    }
    // C < 8: element j of a thread has channel j mod C
    if (C <= 4)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] += part[j + 4];
    if (C <= 2)
#pragma unroll
        for (int j = 0; j < 2; ++j) part[j] += part[j + 2];
    if (C == 1) part[0] += part[1];
    // lanes l and l ^ o hold the same channels when C divides 8 o
    for (int o = 32; o >= 1 && 8 * o >= C; o >>= 1)
#pragma unroll
        for (int j = 0; j < 8; ++j) part[j] += __shfl_xor(part[j], o);
    const int lane = threadIdx.x & 63;
    if (lane < (C >= 8 ? C / 8 : 1))
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < C && part[j] != 0.0f) atomicAdd(&sb[(int)((8 * t0 + j) % (size_t)C)], part[j]);
    __syncthreads();
    if (dbias)
        for (int c = threadIdx.x; c < C; c += blockDim.x)
            if (sb[c] != 0.0f) unsafeAtomicAdd(&dbias[c], sb[c]);
}

__global__ void k_relu_mask(const float* __restrict__ dout, const u16* __restrict__ out, int relu,
                            u16* __restrict__ g, float* __restrict__ dbias, size_t n, int C)
{
    extern __shared__ float sb[];
    for (int c = threadIdx.x; c < C; c += blockDim.x) sb[c] = 0.0f;
    __syncthreads();
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float v = dout[i];
        if (relu && !(bf2f(out[i]) > 0.0f)) v = 0.0f;
        const u16 b = f2bf(v);
        g[i] = b;
        if (v != 0.0f) atomicAdd(&sb[i % C], bf2f(b));
    }
    __syncthreads();
    if (dbias)
        for (int c = threadIdx.x; c < C; c += blockDim.x)
            if (sb[c] != 0.0f) unsafeAtomicAdd(&dbias[c], sb[c]);
}

// Loss 1/V sum (x - t)^2 of the network output (FP32) against the target,
// and its gradient through the final ReLU.
__global__ void k_mse(const float* __restrict__ x, const float* __restrict__ t, float* __restrict__ g,
                      double* __restrict__ loss, size_t n)
{
    __shared__ double red[4];
    double s = 0.0;
    const float inv = 1.0f / (float)n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double dd = (double)x[i] - (double)t[i];   // exact for FP32 inputs
        s += dd * dd;
        const float d = x[i] - t[i];
        g[i] = 2.0f * d * inv;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) / (double)n);
}

// Adam on FP32 master weights (bias-corrected), gradients cleared after use.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        g[i] = 0.0f;
    }
}

// Network input: A^T y scaled by 1 / max (max over the volume), as BF16.
__global__ void k_absmax(const float* __restrict__ x, size_t n, unsigned int* __restrict__ out)
{
    float mval = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        mval = fmaxf(mval, fabsf(x[i]));
    for (int o = 32; o > 0; o >>= 1) mval = fmaxf(mval, __shfl_xor(mval, o));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(mval));
}

__global__ void k_scale_to_bf16(const float* __restrict__ x, const unsigned int* __restrict__ mx,
                                u16* __restrict__ y, size_t n)
{
    const float m = __uint_as_float(*mx);
    const float s = m > 0.0f ? 1.0f / m : 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i] * s);
}

__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        a[i] += b[i];
}

__global__ void k_fill_u32(unsigned int* p, size_t n, unsigned int v)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned nblocks(size_t n)
{
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 16384 ? 16384 : (b ? b : 1));
}

template <int KS, bool CIN1, int NT, int MT>
hipError_t conv_launch(const ConvFwd& a, int groups, hipStream_t s)
{
    const int V = a.D * a.H * a.W;
    const int per_block = 4 * 16 * MT;
    hipLaunchKernelGGL((k_conv_fwd<KS, CIN1, NT, MT>), dim3((V + per_block - 1) / per_block, groups), dim3(256),
                       0, s, a);
    return hipGetLastError();
}

template <int KS, bool CIN1, int NT>
hipError_t conv_mt(const ConvFwd& a, hipStream_t s)
{
    constexpr int MT = NT >= 8 ? 1 : (NT >= 4 ? 2 : 4);
    const int V = a.D * a.H * a.W;
    // small grids (16^3, 32^3): one 16-channel tile and 16 voxels per wave, the
    // channel tiles spread over blockIdx.y, so enough waves run to hide latency
    if (NT > 1 && (long long)(V + 4 * 16 * MT - 1) / (4 * 16 * MT) < 256)
        return conv_launch<KS, CIN1, 1, 1>(a, NT, s);
    return conv_launch<KS, CIN1, NT, MT>(a, 1, s);
}

template <int KS, bool CIN1>
hipError_t conv_nt(const ConvFwd& a, int nt, hipStream_t s)
{
    switch (nt) {
        case 1: return conv_mt<KS, CIN1, 1>(a, s);
        case 2: return conv_mt<KS, CIN1, 2>(a, s);
        case 4: return conv_mt<KS, CIN1, 4>(a, s);
        case 8: return conv_mt<KS, CIN1, 8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t nn_conv_fwd(const ConvFwd& a, int ks, hipStream_t s)
{
    const int nt = (a.cout + 15) / 16;
    const int ntp = nt <= 1 ? 1 : (nt <= 2 ? 2 : (nt <= 4 ? 4 : 8));
    const int cin = a.c0 + a.c1;
    const bool cin1 = cin == 1;
    if (ks == 3 && cin >= 8 && cin <= 64 && cin % 8 == 0) {
        // 8 output planes per workgroup up to 16 channels (35 KiB halo), 4 up to 32
        // (41 KiB), 2 up to 64 (55 KiB)
        const int tz = (cin <= 16 && ntp <= 4) ? 8 : (cin <= 32 ? 4 : 2);
        const dim3 g((a.W + kTX - 1) / kTX, (a.H + kTY - 1) / kTY, (a.D + tz - 1) / tz);
        // the halo, then the per-step offset table (nsteps x 4 ints)
        const size_t lds = (size_t)kHX * kHY * (tz + 2) * cin * sizeof(unsigned short) +
                           (size_t)(a.Kp / 32) * 4 * sizeof(int);
        if (tz == 8) {
            switch (ntp) {
            case 1: hipLaunchKernelGGL((k_conv_fwd_lds<1, 8>), g, dim3(256), lds, s, a); break;
            case 2: hipLaunchKernelGGL((k_conv_fwd_lds<2, 8>), g, dim3(256), lds, s, a); break;
            case 4: hipLaunchKernelGGL((k_conv_fwd_lds<4, 8>), g, dim3(256), lds, s, a); break;
            default: return hipErrorInvalidValue;   // tz = 8 is chosen only for ntp <= 4
            }
        } else if (tz == 4) {
            switch (ntp) {
            case 1: hipLaunchKernelGGL((k_conv_fwd_lds<1, 4>), g, dim3(256), lds, s, a); break;
            case 2: hipLaunchKernelGGL((k_conv_fwd_lds<2, 4>), g, dim3(256), lds, s, a); break;
            case 4: hipLaunchKernelGGL((k_conv_fwd_lds<4, 4>), g, dim3(256), lds, s, a); break;
            default: hipLaunchKernelGGL((k_conv_fwd_lds<8, 4>), g, dim3(256), lds, s, a); break;
            }
        } else {
            switch (ntp) {
            case 1: hipLaunchKernelGGL((k_conv_fwd_lds<1, 2>), g, dim3(256), lds, s, a); break;
            case 2: hipLaunchKernelGGL((k_conv_fwd_lds<2, 2>), g, dim3(256), lds, s, a); break;
            case 4: hipLaunchKernelGGL((k_conv_fwd_lds<4, 2>), g, dim3(256), lds, s, a); break;
            default: hipLaunchKernelGGL((k_conv_fwd_lds<8, 2>), g, dim3(256), lds, s, a); break;
            }
        }
        return hipGetLastError();
    }
    if (ks == 1 && a.cout == 1 && a.c1 == 0 && !a.up && (cin == 8 || cin == 16 || cin == 32)) {
        const size_t nvox = (size_t)a.D * a.H * a.W;
        const dim3 g(std::min(nblocks(nvox), 4096u));
        if (cin == 8) hipLaunchKernelGGL((k_conv1x1_out1<8>), g, dim3(256), 0, s, a, nvox);
        else if (cin == 16) hipLaunchKernelGGL((k_conv1x1_out1<16>), g, dim3(256), 0, s, a, nvox);
        else hipLaunchKernelGGL((k_conv1x1_out1<32>), g, dim3(256), 0, s, a, nvox);
        return hipGetLastError();
    }
    if (ks == 3 && cin1 && a.c1 == 0 && a.cout <= 16) {
        const dim3 g((a.W + 15) / 16, (a.H + 3) / 4, (a.D + 3) / 4);
        hipLaunchKernelGGL(k_conv_fwd_c1, g, dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (ks == 3) return cin1 ? conv_nt<3, true>(a, ntp, s) : conv_nt<3, false>(a, ntp, s);
    return cin1 ? conv_nt<1, true>(a, ntp, s) : conv_nt<1, false>(a, ntp, s);
}

hipError_t nn_conv_wgrad(const ConvWgrad& a, int ks, hipStream_t s)
{
    const int cin = a.c0 + a.c1;
    const int xc = a.W % 128 == 0 ? 128 : a.W % 64 == 0 ? 64 : a.W % 32 == 0 ? 32 : 0;
    if (ks == 3 && xc && cin % 16 == 0 && a.c0 % 8 == 0 && a.cout % 16 == 0 && a.K == 27 * cin &&
        (!a.up || (a.W % 2 == 0 && a.H % 2 == 0 && a.D % 2 == 0))) {
        if (xc == 128) return wgrad_rows<128>(a, s);
        if (xc == 64) return wgrad_rows<64>(a, s);
        return wgrad_rows<32>(a, s);
    }
    if (ks == 3 && cin == 1 && a.c1 == 0 && !a.up && xc && a.cout % 16 == 0 && a.K == 27) {
        if (xc == 128) return wgrad_c1<128>(a, s);
        if (xc == 64) return wgrad_c1<64>(a, s);
        return wgrad_c1<32>(a, s);
    }
    if (ks == 1 && a.cout == 1 && a.c1 == 0 && !a.up && a.K == cin && (cin == 8 || cin == 16 || cin == 32)) {
        const size_t nvox = (size_t)a.D * a.H * a.W;
        const dim3 g(std::min(nblocks(nvox), 1024u));
        if (cin == 8) hipLaunchKernelGGL((k_wgrad_1x1_out1<8>), g, dim3(256), 0, s, a, nvox);
        else if (cin == 16) hipLaunchKernelGGL((k_wgrad_1x1_out1<16>), g, dim3(256), 0, s, a, nvox);
        else hipLaunchKernelGGL((k_wgrad_1x1_out1<32>), g, dim3(256), 0, s, a, nvox);
        return hipGetLastError();
    }
    auto lg2 = [](int n) { int l = 0; while ((1 << l) < n) ++l; return (1 << l) == n ? l : -1; };
    const int lw = lg2(a.W), lh = lg2(a.H);
    if (ks == 3 && lw >= 3 && lh >= 0 && (a.W * a.H) % 32 == 0 && a.cout % 16 == 0 &&
        (!a.up || (a.W % 2 == 0 && a.H % 2 == 0))) {
        constexpr int NK = 2;
        const int tiles = (a.cout / 16) * (((a.K + 15) / 16 + NK - 1) / NK);
        // split each slice's voxel groups over workgroups until ~8192 waves
        // run (one per tile, slice and share); each share adds its own
        // partial sums into dw
        const int blocks = (tiles + 3) / 4 * a.D;
        const int groups = a.W * a.H / 32;
        const int shares = std::max(1, std::min(groups, 2048 / std::max(1, blocks)));
        hipLaunchKernelGGL((k_conv_wgrad_pow2<3, NK>), dim3((tiles + 3) / 4, a.D, shares), dim3(256), 0, s, a,
                           lw, lh);
        return hipGetLastError();
    }
    const int tiles = ((a.cout + 15) / 16) * ((a.K + 15) / 16);
    const int blocks = (tiles + 3) / 4 * a.D;
    const int shares = std::max(1, std::min((a.W * a.H + 31) / 32, 2048 / std::max(1, blocks)));
    dim3 grid((tiles + 3) / 4, a.D, shares);
    if (ks == 3)
        hipLaunchKernelGGL(k_conv_wgrad<3>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_conv_wgrad<1>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t nn_pack(const float* w, int cout, int cin, int taps, unsigned short* wf, int rows_f, int kp_f,
                   unsigned short* wb, int rows_b, int kp_b, hipStream_t s)
{
    const size_t n = (size_t)rows_f * kp_f + (wb ? (size_t)rows_b * kp_b : 0);
    hipLaunchKernelGGL(k_pack, dim3(nblocks(n)), dim3(256), 0, s, w, cout, cin, taps, wf, rows_f, kp_f, wb,
                       rows_b, kp_b);
    return hipGetLastError();
}

hipError_t nn_maxpool(const unsigned short* x, unsigned short* y, unsigned char* arg, int D, int H, int W, int C,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_maxpool, dim3(nblocks((size_t)D * H * W * C / 8)), dim3(256), 0, s, x, y, arg, D, H, W, C);
    return hipGetLastError();
}

hipError_t nn_maxpool_bwd(const float* dy, const unsigned char* arg, float* dx, int D, int H, int W, int C,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_maxpool_bwd, dim3(nblocks((size_t)D * H * W * C / 8)), dim3(256), 0, s, dy, arg, dx, D,
                       H, W, C);
    return hipGetLastError();
}

hipError_t nn_sumpool(const float* dh, float* dl, int D, int H, int W, int C, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_sumpool, dim3(nblocks((size_t)D * H * W * C / 8)), dim3(256), 0, s, dh, dl, D, H, W, C,
                       accumulate);
    return hipGetLastError();
}

hipError_t nn_relu_mask(const float* dout, const unsigned short* out, int relu, unsigned short* g,
                        float* dbias, size_t n, int C, hipStream_t s)
{
    // at most 1024 workgroups: each adds C partial sums into dbias with
    // global atomics, which contend on the C addresses
    const bool pow2 = C >= 1 && (C & (C - 1)) == 0;
    const bool aligned = ((reinterpret_cast<uintptr_t>(dout) | reinterpret_cast<uintptr_t>(out) |
                           reinterpret_cast<uintptr_t>(g)) & 15) == 0;
    if (pow2 && C <= 2048 && n % 8 == 0 && aligned) {   // C divides the grid stride in elements (2048 k)
        hipLaunchKernelGGL(k_relu_mask_v8, dim3(std::min(nblocks(n / 8), 1024u)), dim3(256), C * sizeof(float), s,
                           dout, out, relu, g, dbias, n / 8, C);
        return hipGetLastError();
    }
    const dim3 grid(std::min(nblocks(n), 1024u));
    if (pow2 && C <= 256)   // C divides the grid stride (a multiple of 256)
        hipLaunchKernelGGL(k_relu_mask_pc, grid, dim3(256), C * sizeof(float), s, dout, out, relu, g, dbias, n, C);
    else
        hipLaunchKernelGGL(k_relu_mask, grid, dim3(256), C * sizeof(float), s, dout, out, relu, g, dbias, n, C);
    return hipGetLastError();
}

hipError_t nn_mse(const float* x, const float* t, float* g, double* loss, size_t n, hipStream_t s)
{
    // at most 1024 workgroups: each adds its partial loss with one FP64 atomic
    hipLaunchKernelGGL(k_mse, dim3(std::min(nblocks(n), 1024u)), dim3(256), 0, s, x, t, g, loss, n);
    return hipGetLastError();
}

hipError_t nn_adam(float* w, float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                   int step, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t nn_prep_input(const float* x, unsigned short* y, unsigned int* scratch, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, scratch, (size_t)1, 0u);
    hipLaunchKernelGGL(k_absmax, dim3(std::min(nblocks(n), 1024u)), dim3(256), 0, s, x, n, scratch);
    hipLaunchKernelGGL(k_scale_to_bf16, dim3(nblocks(n)), dim3(256), 0, s, x, scratch, y, n);
    return hipGetLastError();
}

hipError_t nn_add(float* a, const float* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

}  // namespace ltm
