// cnn.hip -- kernels of the learned refinement-flag predictor (include/lbm_cnn.h).
//
// 3x3x3 "same" convolutions over channels-last float32 activations, as
// implicit GEMMs on the gfx950 matrix cores: v_mfma_f32_16x16x16_bf16 takes a
// 16x16 bfloat16 A tile and a 16x16 bfloat16 B tile spread over the 64 lanes
// of a wave (lane i holds row i%16, reduction entries 4*(i/16)..+3 of A and
// the transposed arrangement of B) and accumulates a 16x16 float32 tile
// (lane i holds rows 4*(i/16)..+3 of column i%16).
//  * forward: rows = 16 consecutive voxels, columns = 16 output channels,
//    reduction = (tap, input channel), with the input gathered on the fly
//    (zero outside the grid);
//  * data gradient: the forward kernel applied to the output gradient with
//    mirrored taps and transposed channels (packed by lbm_cnn_pack_weights);
//  * weight gradient: rows = 16 output channels, columns = 16 (tap, input
//    channel) pairs, reduction = voxels, per-workgroup partials folded in a
//    fixed order.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "lbm_cnn.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTaps = 27;
constexpr int kWgradVoxels = 512;    // voxels per weight-gradient workgroup
constexpr int kLossBlocks = 256;     // workgroups of the loss kernel (partial sums in loss[1..])

__host__ __device__ inline int pad4(int c) { return (c + 3) / 4 * 4; }
__host__ __device__ inline int pad16(int k) { return (k + 15) / 16 * 16; }

__device__ inline short to_bf16(float v) {
    return __builtin_bit_cast(short, static_cast<__bf16>(v));   // round to nearest even
}

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));

// Four floats to bfloat16 (round to nearest even), two per packed conversion.
__device__ inline bf16x4 to_bf16x4(float a, float b, float c, float d) {
    const bf16x2v lo = __builtin_convertvector((f32x2v){a, b}, bf16x2v);
    const bf16x2v hi = __builtin_convertvector((f32x2v){c, d}, bf16x2v);
    const unsigned u[2] = {__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
    return __builtin_bit_cast(bf16x4, u);
}

struct Vox {
    int n, z, y, x;
};

__device__ inline Vox decompose(int v, int d, int h, int w) {
    Vox r;
    r.x = v % w;
    r.y = (v / w) % h;
    r.z = (v / (w * h)) % d;
    r.n = v / (w * h * d);
    return r;
}

// Index of the voxel at tap offset from p, or -1 outside the grid.
__device__ inline int64_t tap_voxel(const Vox &p, int tap, int d, int h, int w) {
    const int zz = p.z + tap / 9 - 1, yy = p.y + (tap / 3) % 3 - 1, xx = p.x + tap % 3 - 1;
    if (zz < 0 || yy < 0 || xx < 0 || zz >= d || yy >= h || xx >= w) return -1;
    return (((int64_t)p.n * d + zz) * h + yy) * w + xx;
}

__global__ void pack_kernel(const float *w, int co, int ci, int flip, uint16_t *out, int rows16, int k16) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows16 * k16) return;
    const int row = idx / k16, k = idx % k16;
    float v = 0.0f;
    if (!flip) {
        const int ci4 = pad4(ci), tap = k / ci4, c = k % ci4;
        if (row < co && tap < kTaps && c < ci) v = w[((int64_t)row * kTaps + tap) * ci + c];
    } else {
        const int co4 = pad4(co), tap = k / co4, o = k % co4;
        if (row < ci && tap < kTaps && o < co) v = w[((int64_t)o * kTaps + (kTaps - 1 - tap)) * ci + row];
    }
    out[idx] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}

// Bias, ReLU, mask and store of a forward output tile: lane (r, kg) holds
// voxels v0 + 4 kg .. + 3 of output channel co0 + r.
__device__ __forceinline__ void store_tile(const f32x4 &acc, int v0, int nv, int co0, int r, int kg, int co,
                                           int co4, const float *bias, int relu, const float *mask, float *y) {
    const int oc = co0 + r;
    if (oc >= co4) return;
    const float b = (bias && oc < co) ? bias[oc] : 0.0f;
    // the mask values of the 4 voxels loaded together (a load inside the
    // store loop had been waited for voxel by voxel)
    float mv[4] = {1.0f, 1.0f, 1.0f, 1.0f};
    if (mask) {
#pragma unroll
        for (int j = 0; j < 4; ++j) mv[j] = mask[(int64_t)min(v0 + 4 * kg + j, nv - 1) * co4 + oc];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = v0 + 4 * kg + j;
        if (v >= nv) continue;
        float o = acc[j] + b;
        if (relu) o = o > 0.0f ? o : 0.0f;
        if (mask) o = mv[j] > 0.0f ? o : 0.0f;
        y[(int64_t)v * co4 + oc] = o;
    }
}

// One wave: 16 voxels x 16 output channels.  Four waves per workgroup, no
// barriers, so a wave past the last voxel simply returns.
__global__ __launch_bounds__(256) void conv_forward_kernel(const float *x, int n, int d, int h, int w, int ci,
                                                           const uint16_t *packed, int co, const float *bias,
                                                           int relu, const float *mask, float *y) {
    const int ci4 = pad4(ci), co4 = pad4(co), k16 = pad16(kTaps * ci4);
    const int nv = n * d * h * w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int v0 = (blockIdx.x * 4 + wave) * 16;
    const int co0 = blockIdx.y * 16;
    if (v0 >= nv) return;
    const int r = lane & 15, kg = lane >> 4;
    const int va = v0 + r;
    const Vox pa = decompose(va < nv ? va : 0, d, h, w);
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    // nine K steps per pass (27 taps of 16 channels in three passes): their
    // loads (each from a clamped, always valid index, zeroed by a select) are
    // issued before their MFMAs, which run in step order
    constexpr int kPass = 9;
    const uint16_t *wrow = packed + (int64_t)(co0 + r) * k16;
    for (int kc0 = 0; kc0 < k16; kc0 += 16 * kPass) {
        float4 a[kPass];
        bf16x4 B[kPass];
#pragma unroll
        for (int q = 0; q < kPass; ++q) {
            const int k = kc0 + 16 * q + 4 * kg;
            const int tap = k / ci4, c = k % ci4;   // 4 consecutive k share the tap
            const int64_t src = (va < nv && k < k16 && tap < kTaps) ? tap_voxel(pa, tap, d, h, w) : -1;
            a[q] = *reinterpret_cast<const float4 *>(x + (src >= 0 ? src * ci4 + c : 0));
            if (src < 0) a[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            B[q] = *reinterpret_cast<const bf16x4 *>(wrow + (k < k16 ? k : 0));
        }
#pragma unroll
        for (int q = 0; q < kPass; ++q)
            if (kc0 + 16 * q < k16)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(to_bf16x4(a[q].x, a[q].y, a[q].z, a[q].w), B[q],
                                                                acc, 0, 0, 0);
    }
    store_tile(acc, v0, nv, co0, r, kg, co, co4, bias, relu, mask, y);
}

// The same convolution for 4 or 16 (padded) input channels, the
// predictor's: with CI a compile-time constant, the tap of K step s is s
// itself (CI = 16) or 4 s + lane group (CI = 4), so its neighbour offset and
// its bounds test come from the lane's voxel, decomposed once, instead of a
// division and a 64-bit index per step; a step's source is the lane's base
// pointer plus the tap's offset.  (The generic kernel spends ~30 VALU per
// MFMA on that index arithmetic.)  The same operands in the same order as
// conv_forward_kernel: the same bits.
// (Workgroup (bx, by) of the launch: voxel tiles 4 bx .. 4 bx + 3, output
// channels 16 by ..; a body of its own so that a fused launch can run it.)

// WAVES waves per workgroup, one 16-voxel tile each (8 in conv_forward_ci, 4
// in the data-gradient part of backward_layer_kernel).
template <int CI, int WAVES = 4>
__device__ __forceinline__ void conv_forward_ci_body(const float *x, int n, int d, int h, int w,
                                                     const uint16_t *packed, int co, const float *bias, int relu,
                                                     const float *mask, float *y, int bx, int by) {
    constexpr int K16 = (kTaps * CI + 15) / 16 * 16, NK = K16 / 16;
    const int co4 = pad4(co);
    const int nv = n * d * h * w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int v0 = (bx * WAVES + wave) * 16;
    const int co0 = by * 16;
    // the workgroup's weight operands, the same for all its tiles, staged once
    // in LDS ([K step][lane], the lane layout of the MFMA operand) before any
    // wave may leave
    __shared__ bf16x4 wsh[NK * 64];
    for (int e = threadIdx.x; e < NK * 64; e += 64 * WAVES) {
        const int l = e & 63;
        wsh[e] = *reinterpret_cast<const bf16x4 *>(packed + (int64_t)(co0 + (l & 15)) * K16 + 16 * (e >> 6) +
                                                   4 * (l >> 4));
    }
    __syncthreads();
    if (v0 >= nv) return;
    const int r = lane & 15, kg = lane >> 4;
    const int va = v0 + r;
    const bool vok = va < nv;
    const Vox pa = decompose(vok ? va : 0, d, h, w);
    // is the neighbour at offset -1, 0, +1 along each axis inside the grid
    const bool zok[3] = {pa.z > 0, true, pa.z < d - 1};
    const bool yok[3] = {pa.y > 0, true, pa.y < h - 1};
    const bool xok[3] = {pa.x > 0, true, pa.x < w - 1};
    const int hw = h * w;
    const float *xb = x + (int64_t)(vok ? va : 0) * CI + (CI == 16 ? 4 * kg : 0);
    const bf16x4 *B = wsh + lane;   // B[64 s]: the weight operand of K step s
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (CI == 16) {
        if (w == 16) {
            // A tile's 16 voxels are one whole grid row (v0 is a multiple of
            // 16 = w), lane r holding x = r.  The taps 3g, 3g + 1, 3g + 2 of
            // one (z, y) offset read the same row of the input shifted by x
            // offsets -1, 0, +1, and a shift of one voxel is a shift of one
            // lane within each 16-lane row of the operand: load the 9 rows
            // once and form the other two taps' operands with DPP row shifts
            // (zero where the shift leaves the row: x = -1 or 16, outside
            // the grid).  The operands, and so the bits, are those of the
            // general loop below.  (A row past nv cannot occur: nv is a
            // multiple of 16.)
            float4 a[9];
            bool rok[9];
#pragma unroll
            for (int g = 0; g < 9; ++g) {
                const int dz = g / 3, dy = g % 3;
                rok[g] = vok && zok[dz] && yok[dy];
                const int off = ((dz - 1) * hw + (dy - 1) * w) * CI;
                a[g] = *reinterpret_cast<const float4 *>(xb + (rok[g] ? off : 0));
            }
#pragma unroll
            for (int g = 0; g < 9; ++g) {
                const bf16x4 zero = {0, 0, 0, 0};
                const bf16x4 A = rok[g] ? to_bf16x4(a[g].x, a[g].y, a[g].z, a[g].w) : zero;
                const int2 ai = __builtin_bit_cast(int2, A);
                // row_shr:1 (lane r takes lane r - 1) and row_shl:1 (lane r + 1), 0 at the row's end
                const int2 lo = {__builtin_amdgcn_update_dpp(0, ai.x, 0x111, 0xF, 0xF, true),
                                 __builtin_amdgcn_update_dpp(0, ai.y, 0x111, 0xF, 0xF, true)};
                const int2 hi = {__builtin_amdgcn_update_dpp(0, ai.x, 0x101, 0xF, 0xF, true),
                                 __builtin_amdgcn_update_dpp(0, ai.y, 0x101, 0xF, 0xF, true)};
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, lo), B[64 * (3 * g)], acc,
                                                                0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B[64 * (3 * g + 1)], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, hi), B[64 * (3 * g + 2)],
                                                                acc, 0, 0, 0);
            }
            store_tile(acc, v0, nv, co0, r, kg, co, co4, bias, relu, mask, y);
            return;
        }
    }
    constexpr int kPass = 9;
#pragma unroll
    for (int s0 = 0; s0 < NK; s0 += kPass) {
        float4 a[kPass];
        bool ok[kPass];
#pragma unroll
        for (int q = 0; q < kPass; ++q) {
            const int s = s0 + q;
            if (s < NK) {
                const int tap = (CI == 16) ? s : 4 * s + kg;   // k = 16 s + 4 kg, tap = k / CI
                const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // offsets + 1
                ok[q] = vok && tap < kTaps && zok[dz] && yok[dy] && xok[dx];
                const int off = ((dz - 1) * hw + (dy - 1) * w + (dx - 1)) * CI;
                a[q] = *reinterpret_cast<const float4 *>(xb + (ok[q] ? off : 0));
            }
        }
#pragma unroll
        for (int q = 0; q < kPass; ++q)
            if (s0 + q < NK) {
                // outside the grid: zeros (the load above read the lane's own voxel)
                const bf16x4 A = to_bf16x4(a[q].x, a[q].y, a[q].z, a[q].w);
                const bf16x4 zero = {0, 0, 0, 0};
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ok[q] ? A : zero, B[64 * (s0 + q)], acc, 0, 0, 0);
            }
    }
    store_tile(acc, v0, nv, co0, r, kg, co, co4, bias, relu, mask, y);
}

// Weight gradient partials.  Workgroup (chunk, kt, ct): output channels
// 16*ct.., reduction columns 16*kt.. over the chunk's voxels; each wave takes a
// quarter of the voxels, the four wave tiles are summed in LDS in a fixed
// order into work[chunk][co][k].  The workgroups of column tile 0 also sum
// the float32 output gradient per channel (the bias gradient) into
// work[nchunk * co16 * k16 + chunk * co16 + co].
__global__ __launch_bounds__(256) void conv_wgrad_kernel(const float *x, const float *gz, int n, int d, int h,
                                                         int w, int ci, int co, float *work) {
    const int ci4 = pad4(ci), co4 = pad4(co), k16 = pad16(kTaps * ci4), co16 = pad16(co);
    const int nv = n * d * h * w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int chunk = blockIdx.x, k0 = blockIdx.y * 16, c0 = blockIdx.z * 16;
    const int r = lane & 15, kg = lane >> 4;
    const int kcol = k0 + r;                       // this lane's B column
    const int tap = kcol / ci4, cch = kcol % ci4;
    const bool col_ok = tap < kTaps && cch < ci;
    const int ocol = c0 + r;                       // this lane's A row (output channel)
    const bool row_ok = ocol < co;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    const int vbeg = chunk * kWgradVoxels + wave * (kWgradVoxels / 4);
    const int vend = min(vbeg + kWgradVoxels / 4, nv);
    // The lane's tap offset is fixed; its 4 voxels v0 + 4 kg + j are
    // consecutive and, when w is a multiple of 4, lie in one row (v0 is a
    // multiple of 16), so one decomposition per step serves all four.
    const int tdz = tap / 9 - 1, tdy = (tap / 3) % 3 - 1, tdx = tap % 3 - 1;
    const int tdelta = (tdz * h + tdy) * w + tdx;
    const bool rows4 = (w & 3) == 0;
    auto step = [&](const float (&a)[4], const float (&b)[4]) {
        bsum += ((a[0] + a[1]) + a[2]) + a[3];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(to_bf16x4(a[0], a[1], a[2], a[3]),
                                                        to_bf16x4(b[0], b[1], b[2], b[3]), acc, 0, 0, 0);
    };
    if (rows4) {
        // four steps per pass: the loads of all four are issued before their
        // MFMAs (each from a clamped, always valid index, zeroed by a select),
        // so a wave keeps 32 loads in flight; the sums run in step order
        constexpr int kPass = 4;
        for (int v0 = vbeg; v0 < vend; v0 += 16 * kPass) {
            float a[kPass][4], b[kPass][4];
#pragma unroll
            for (int q = 0; q < kPass; ++q) {
                const int vq = v0 + 16 * q + 4 * kg;
                const Vox p = decompose(vq < nv ? vq : 0, d, h, w);
                const bool zy_ok = col_ok && p.z + tdz >= 0 && p.z + tdz < d && p.y + tdy >= 0 && p.y + tdy < h;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int v = vq + j;
                    const int xx = p.x + j + tdx;
                    const bool oka = v < vend && row_ok;
                    const bool okb = v < vend && zy_ok && xx >= 0 && xx < w;
                    const float av = gz[oka ? (int64_t)v * co4 + ocol : 0];
                    const float bv = x[okb ? (int64_t)(v + tdelta) * ci4 + cch : 0];
                    a[q][j] = oka ? av : 0.0f;
                    b[q][j] = okb ? bv : 0.0f;
                }
            }
#pragma unroll
            for (int q = 0; q < kPass; ++q)
                if (v0 + 16 * q < vend) step(a[q], b[q]);
        }
    } else {
        for (int v0 = vbeg; v0 < vend; v0 += 16) {
            float a[4], b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int v = v0 + 4 * kg + j;
                a[j] = 0.0f;
                b[j] = 0.0f;
                if (v < vend) {
                    if (row_ok) a[j] = gz[(int64_t)v * co4 + ocol];
                    if (col_ok) {
                        const int64_t src = tap_voxel(decompose(v, d, h, w), tap, d, h, w);
                        if (src >= 0) b[j] = x[src * ci4 + cch];
                    }
                }
            }
            step(a, b);
        }
    }
    __shared__ float tile[4][16][16];
    __shared__ float bias[4][4][16];   // [wave][lane group][channel]
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[wave][4 * kg + j][r] = acc[j];
    bias[wave][kg][r] = bsum;
    __syncthreads();
    const int t = threadIdx.x;   // 256 threads = one 16x16 tile
    const int row = t / 16, col = t % 16;
    const float s = ((tile[0][row][col] + tile[1][row][col]) + tile[2][row][col]) + tile[3][row][col];
    work[((int64_t)chunk * co16 + c0 + row) * k16 + k0 + col] = s;
    if (blockIdx.y == 0 && t < 16) {
        float b = 0.0f;
        for (int wv = 0; wv < 4; ++wv)
            for (int g = 0; g < 4; ++g) b += bias[wv][g][t];
        work[(int64_t)gridDim.x * co16 * k16 + (int64_t)chunk * co16 + c0 + t] = b;
    }
}

template <int CI>
__global__ __launch_bounds__(512) void conv_forward_ci(const float *x, int n, int d, int h, int w,
                                                       const uint16_t *packed, int co, const float *bias,
                                                       int relu, const float *mask, float *y) {
    conv_forward_ci_body<CI, 8>(x, n, d, h, w, packed, co, bias, relu, mask, y, blockIdx.x, blockIdx.y);
}

// The same weight-gradient partials for 4 or 16 (padded) input channels and
// rows of a multiple of 4 voxels: the lane's first voxel is decomposed once
// and then advanced by 16 voxels per step (carrying into y, z, n), its
// gradient and input pointers by 16 voxels' strides, so a step is its
// bounds tests, eight loads and one MFMA.  The same operands in the same
// order as conv_wgrad_kernel: the same bits.
// (Workgroup (chunk, bk, bc) of nchunk chunks: a body of its own so that a
// fused launch can run it.)
template <int CI>
__device__ __forceinline__ void conv_wgrad_ci_body(const float *x, const float *gz, int n, int d, int h, int w,
                                                   int ci, int co, float *work, int chunk, int bk, int bc,
                                                   int nchunk) {
    constexpr int K16 = (kTaps * CI + 15) / 16 * 16;
    const int co4 = pad4(co), co16 = pad16(co);
    const int nv = n * d * h * w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k0 = bk * 16, c0 = bc * 16;
    const int r = lane & 15, kg = lane >> 4;
    const int kcol = k0 + r;                       // this lane's B column
    const int tap = kcol / CI, cch = kcol % CI;
    const bool col_ok = tap < kTaps && cch < ci;
    const int ocol = c0 + r;                       // this lane's A row (output channel)
    const bool row_ok = ocol < co;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    const int vbeg = chunk * kWgradVoxels + wave * (kWgradVoxels / 4);
    const int vend = min(vbeg + kWgradVoxels / 4, nv);
    const int tdz = tap / 9 - 1, tdy = (tap / 3) % 3 - 1, tdx = tap % 3 - 1;
    const int tdelta = (tdz * h + tdy) * w + tdx;
    // the lane's 4 voxels of step 0: vq .. vq + 3, one row (w is a multiple of 4)
    int vq = vbeg + 4 * kg;
    Vox p = decompose(vq < nv ? vq : 0, d, h, w);
    const float *gp = gz + (int64_t)vq * co4 + ocol;
    const float *xp = x + ((int64_t)vq + tdelta) * CI + cch;
    auto step = [&](const float (&a)[4], const float (&b)[4]) {
        bsum += ((a[0] + a[1]) + a[2]) + a[3];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(to_bf16x4(a[0], a[1], a[2], a[3]),
                                                        to_bf16x4(b[0], b[1], b[2], b[3]), acc, 0, 0, 0);
    };
    constexpr int kPass = 4;
    for (int v0 = vbeg; v0 < vend; v0 += 16 * kPass) {
        float a[kPass][4], b[kPass][4];
#pragma unroll
        for (int q = 0; q < kPass; ++q) {
            const bool zy_ok = col_ok && p.z + tdz >= 0 && p.z + tdz < d && p.y + tdy >= 0 && p.y + tdy < h;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int v = vq + j;
                const int xx = p.x + j + tdx;
                const bool oka = v < vend && row_ok;
                const bool okb = v < vend && zy_ok && xx >= 0 && xx < w;
                const float av = *(oka ? gp + j * co4 : gz);
                const float bv = *(okb ? xp + j * CI : x);
                a[q][j] = oka ? av : 0.0f;
                b[q][j] = okb ? bv : 0.0f;
            }
            // the next 16 voxels
            vq += 16;
            gp += 16 * co4;
            xp += 16 * CI;
            p.x += 16;
            while (p.x >= w) {
                p.x -= w;
                if (++p.y == h) {
                    p.y = 0;
                    if (++p.z == d) p.z = 0;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kPass; ++q)
            if (v0 + 16 * q < vend) step(a[q], b[q]);
    }
    __shared__ float tile[4][16][16];
    __shared__ float bias[4][4][16];   // [wave][lane group][channel]
#pragma unroll
    for (int j = 0; j < 4; ++j) tile[wave][4 * kg + j][r] = acc[j];
    bias[wave][kg][r] = bsum;
    __syncthreads();
    const int t = threadIdx.x;   // 256 threads = one 16x16 tile
    const int row = t / 16, col = t % 16;
    const float sum = ((tile[0][row][col] + tile[1][row][col]) + tile[2][row][col]) + tile[3][row][col];
    work[((int64_t)chunk * co16 + c0 + row) * K16 + k0 + col] = sum;
    if (bk == 0 && t < 16) {
        float bb = 0.0f;
        for (int wv = 0; wv < 4; ++wv)
            for (int g = 0; g < 4; ++g) bb += bias[wv][g][t];
        work[(int64_t)nchunk * co16 * K16 + (int64_t)chunk * co16 + c0 + t] = bb;
    }
}

// The weight gradient for 16 (padded) input channels, three taps per
// workgroup: the taps 3g, 3g + 1, 3g + 2 of one (z, y) offset, whose x
// offsets are -1, 0, +1 (reduction columns 16 * tap .. + 15).  They share the
// output-gradient operand, and their input operands are three overlapping
// windows of one row, so a lane loads the gradient once and the 6 input
// voxels x - 1 .. x + 4 of its channel once: 10 loads per voxel group
// instead of 24 with one workgroup per tap (conv_wgrad_ci_body).  Each tap's
// accumulation takes the same voxels, operands and order as there, so the
// partials are the same bits; grid (nchunk, 9, co16 / 16).
__device__ __forceinline__ void conv_wgrad_x3_body(const float *x, const float *gz, int n, int d, int h, int w,
                                                   int ci, int co, float *work, int chunk, int g, int bc,
                                                   int nchunk) {
    constexpr int CI = 16, K16 = kTaps * CI;
    const int co4 = pad4(co), co16 = pad16(co);
    const int nv = n * d * h * w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c0 = bc * 16;
    const int r = lane & 15, kg = lane >> 4;
    const bool col_ok = r < ci;                    // this lane's B column: input channel r
    const int ocol = c0 + r;                       // this lane's A row (output channel)
    const bool row_ok = ocol < co;
    const int tdz = g / 3 - 1, tdy = g % 3 - 1;
    f32x4 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    const int vbeg = chunk * kWgradVoxels + wave * (kWgradVoxels / 4);
    const int vend = min(vbeg + kWgradVoxels / 4, nv);
    // the lane's 4 voxels of step 0: vq .. vq + 3, one row (w is a multiple of 4)
    int vq = vbeg + 4 * kg;
    Vox p = decompose(vq < nv ? vq : 0, d, h, w);
    const float *gp = gz + (int64_t)vq * co4 + ocol;
    const float *xp = x + ((int64_t)vq + (tdz * h + tdy) * w - 1) * CI + r;   // voxel x - 1 of the row
    constexpr int kPass = 4;
    for (int v0 = vbeg; v0 < vend; v0 += 16 * kPass) {
        float a[kPass][4], b[kPass][6];
#pragma unroll
        for (int q = 0; q < kPass; ++q) {
            // a group of 4 voxels lies wholly before vend or wholly after it
            const bool vok = vq < vend;
            const bool zy_ok = vok && col_ok && p.z + tdz >= 0 && p.z + tdz < d && p.y + tdy >= 0 && p.y + tdy < h;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool oka = vok && row_ok;
                const float av = *(oka ? gp + j * co4 : gz);
                a[q][j] = oka ? av : 0.0f;
            }
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const int xx = p.x + m - 1;
                const bool okb = zy_ok && xx >= 0 && xx < w;
                const float bv = *(okb ? xp + m * CI : x);
                b[q][m] = okb ? bv : 0.0f;
            }
            // the next 16 voxels
            vq += 16;
            gp += 16 * co4;
            xp += 16 * CI;
            p.x += 16;
            while (p.x >= w) {
                p.x -= w;
                if (++p.y == h) {
                    p.y = 0;
                    if (++p.z == d) p.z = 0;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kPass; ++q)
            if (v0 + 16 * q < vend) {
                bsum += ((a[q][0] + a[q][1]) + a[q][2]) + a[q][3];
                const bf16x4 A = to_bf16x4(a[q][0], a[q][1], a[q][2], a[q][3]);
#pragma unroll
                for (int t = 0; t < 3; ++t)   // x offset t - 1: voxels j + t - 1 of the window
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                        A, to_bf16x4(b[q][t], b[q][t + 1], b[q][t + 2], b[q][t + 3]), acc[t], 0, 0, 0);
            }
    }
    __shared__ float tile[3][4][16][16];
    __shared__ float bias[4][4][16];   // [wave][lane group][channel]
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) tile[t][wave][4 * kg + j][r] = acc[t][j];
    bias[wave][kg][r] = bsum;
    __syncthreads();
    const int t = threadIdx.x;   // 256 threads = one 16x16 tile
    const int row = t / 16, col = t % 16;
#pragma unroll
    for (int tt = 0; tt < 3; ++tt) {
        const float sum = ((tile[tt][0][row][col] + tile[tt][1][row][col]) + tile[tt][2][row][col]) +
                          tile[tt][3][row][col];
        work[((int64_t)chunk * co16 + c0 + row) * K16 + (3 * g + tt) * 16 + col] = sum;
    }
    if (g == 0 && t < 16) {
        float bb = 0.0f;
        for (int wv = 0; wv < 4; ++wv)
            for (int q = 0; q < 4; ++q) bb += bias[wv][q][t];
        work[(int64_t)nchunk * co16 * K16 + (int64_t)chunk * co16 + c0 + t] = bb;
    }
}

__global__ __launch_bounds__(256) void conv_wgrad_x3(const float *x, const float *gz, int n, int d, int h, int w,
                                                     int ci, int co, float *work) {
    conv_wgrad_x3_body(x, gz, n, d, h, w, ci, co, work, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x);
}

template <int CI>
__global__ __launch_bounds__(256) void conv_wgrad_ci(const float *x, const float *gz, int n, int d, int h, int w,
                                                     int ci, int co, float *work) {
    conv_wgrad_ci_body<CI>(x, gz, n, d, h, w, ci, co, work, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x);
}

// One layer's backward in one launch: the weight-gradient partials of the
// layer (input x with ci channels, output gradient gz with co) and its data
// gradient (the forward body with flip-packed weights, gz -> gin with ci
// channels, masked by the ReLU of the layer below); the first nwg
// workgroups take the former, the rest the latter.  The two read the same
// gz and write different buffers, so the result is that of the two
// launches.  CIW = ci padded to 4, CIF = co padded to 4.
template <int CIW, int CIF>
__global__ __launch_bounds__(256) void backward_layer_kernel(const float *x, const float *gz, int n, int d, int h,
                                                             int w, int ci, int co, float *work, int nchunk,
                                                             int nk, int nc, const uint16_t *packed_flip,
                                                             const float *mask, float *gin, int fx) {
    const int nwg = nchunk * nk * nc;
    const int b = blockIdx.x;
    if (b < nwg) {
        if constexpr (CIW == 16)   // nk = 9 groups of three taps
            conv_wgrad_x3_body(x, gz, n, d, h, w, ci, co, work, b % nchunk, (b / nchunk) % nk, b / (nchunk * nk),
                               nchunk);
        else
            conv_wgrad_ci_body<CIW>(x, gz, n, d, h, w, ci, co, work, b % nchunk, (b / nchunk) % nk,
                                    b / (nchunk * nk), nchunk);
    } else {
        const int f = b - nwg;
        conv_forward_ci_body<CIF>(gz, n, d, h, w, packed_flip, ci, nullptr, 0, mask, gin, f % fx, f / fx);
    }
}

// The folds, in one launch: gw[co][tap][ci] and (with gb) gb[co] are the
// sums over chunks of the partials.  A workgroup folds 64 outputs (indices
// below co * 27 * ci: weights, the next co: biases) with its 8 waves: wave
// s sums chunks s, s + 8, s + 16, ... in that order, and the 8 sums are
// added pairwise, ((0+1)+(2+3))+((4+5)+(6+7)): a fixed order, so the result
// is deterministic, with 8 loads per lane in flight instead of a chain of
// nchunk.
constexpr int kFoldWaves = 8;
// The fold of output block * 64 + lane (with_bias: biases included); valid
// in wave 0, whose lanes return the sums; ok tells whether the lane's output
// exists.
__device__ inline float fold_output(const float *work, int nchunk, int ci, int co, bool with_bias, bool &ok,
                                    int block) {
    const int ci4 = pad4(ci), k16 = pad16(kTaps * ci4), co16 = pad16(co);
    const int nw = co * kTaps * ci;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int idx = block * 64 + lane;
    const bool is_w = idx < nw, is_b = !is_w && with_bias && idx < nw + co;
    // partial of chunk ch for this output: base + ch * stride
    int64_t base = 0, stride = 0;
    if (is_w) {
        const int c = idx % ci, tap = (idx / ci) % kTaps, o = idx / (ci * kTaps);
        base = (int64_t)o * k16 + tap * ci4 + c;
        stride = (int64_t)co16 * k16;
    } else if (is_b) {
        base = (int64_t)nchunk * co16 * k16 + (idx - nw);
        stride = co16;
    }
    float s = 0.0f;
    if (is_w || is_b) {
#pragma unroll 8
        for (int ch = wave; ch < nchunk; ch += kFoldWaves) s += work[base + ch * stride];
    }
    __shared__ float part[kFoldWaves][64];
    part[wave][lane] = s;
    __syncthreads();
    ok = is_w || is_b;
    return ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) +
           ((part[4][lane] + part[5][lane]) + (part[6][lane] + part[7][lane]));
}

__global__ __launch_bounds__(64 * kFoldWaves) void grad_fold_kernel(const float *work, int nchunk, int ci, int co,
                                                                    float *gw, float *gb) {
    bool ok;
    const float t = fold_output(work, nchunk, ci, co, gb != nullptr, ok, blockIdx.x);
    if (threadIdx.x >= 64 || !ok) return;
    const int nw = co * kTaps * ci, idx = blockIdx.x * 64 + threadIdx.x;
    if (idx < nw) gw[idx] = t;
    else gb[idx - nw] = t;
}


__global__ void relu_backward_kernel(const float *a, float *g, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && !(a[i] > 0.0f)) g[i] = 0.0f;
}

// Squared errors of channel 0 and the output gradient; workgroup b writes
// its partial sum of squares to loss[1 + b] (fixed-order tree).
__global__ __launch_bounds__(256) void mse_kernel(const float *y, int ys, const float *t, int64_t count, float *g,
                                                  float *loss) {
    __shared__ float sh[256];
    float s = 0.0f;
    const float scale = 2.0f / (float)count;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < count; v += (int64_t)gridDim.x * 256) {
        const float e = y[v * ys] - t[v];
        s += e * e;
        g[v * ys] = scale * e;
        for (int c = 1; c < ys; ++c) g[v * ys + c] = 0.0f;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[1 + blockIdx.x] = sh[0];
}

// loss[0] = (sum of the nblocks <= 256 partials) / count, the partials
// added by a fixed pairwise tree (the same order on every call).
__global__ __launch_bounds__(kLossBlocks) void mse_fold_kernel(float *loss, int nblocks, int64_t count) {
    __shared__ float sh[kLossBlocks];
    const int t = threadIdx.x;
    sh[t] = t < nblocks ? loss[1 + t] : 0.0f;
    __syncthreads();
    for (int k = kLossBlocks / 2; k > 0; k >>= 1) {
        if (t < k) sh[t] += sh[t + k];
        __syncthreads();
    }
    if (t == 0) loss[0] = sh[0] / (float)count;
}

__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int64_t count, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// The device-resident form: hyper = {lr, beta1, beta2, eps, t}; the bias
// corrections 1 - beta^t are formed on the device.
__global__ void adam_dev_kernel(float *w, const float *g, float *m, float *v, int64_t count, const float *hyper) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float lr = hyper[0], b1 = hyper[1], b2 = hyper[2], eps = hyper[3], t = hyper[4];
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__device__ inline uint16_t to_bf16_bits(float v) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)); }

// Adam (device hyperparameters) over a layer's weights [co][27][ci] and bias
// [co] in one launch, the arithmetic of adam_dev_kernel; each updated weight
// is also written to both packed forms (the layouts of pack_kernel with flip
// 0 and 1), whose padding entries stay as they are.
// The Adam step of parameter idx of a layer (weights [co][27][ci] first, then
// the co biases) with gradient gi, and the packed BF16 copies of a weight.
__device__ inline void adam_layer_param(int idx, float gi, float *w, float *b, float *mw, float *vw, float *mb,
                                        float *vb, int co, int ci, uint16_t *packed, uint16_t *packed_flip,
                                        const float *hyper) {
    const int nw = co * kTaps * ci;
    const float lr = hyper[0], b1 = hyper[1], b2 = hyper[2], eps = hyper[3], t = hyper[4];
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    const bool is_w = idx < nw;
    const int i = is_w ? idx : idx - nw;
    float *p = is_w ? w : b;
    float *m = is_w ? mw : mb;
    float *v = is_w ? vw : vb;
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pn;
    if (is_w) {
        const int c = i % ci, tap = (i / ci) % kTaps, o = i / (ci * kTaps);
        const int ci4 = pad4(ci), co4 = pad4(co);
        const int k16 = pad16(kTaps * ci4), k16f = pad16(kTaps * co4);
        packed[(int64_t)o * k16 + tap * ci4 + c] = to_bf16_bits(pn);
        packed_flip[(int64_t)c * k16f + (kTaps - 1 - tap) * co4 + o] = to_bf16_bits(pn);
    }
}

__global__ void adam_layer_kernel(float *w, float *b, const float *gw, const float *gb, float *mw, float *vw,
                                  float *mb, float *vb, int co, int ci, uint16_t *packed, uint16_t *packed_flip,
                                  const float *hyper) {
    const int nw = co * kTaps * ci;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nw + co) return;
    const float gi = idx < nw ? gw[idx] : gb[idx - nw];
    adam_layer_param(idx, gi, w, b, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper);
}

// The fold and the Adam step of a layer in one launch: wave 0 of each
// workgroup applies Adam to the 64 sums it folded (the same sums, and the
// same update, as grad_fold_kernel followed by adam_layer_kernel; gw, gb
// receive the gradient when given).
__device__ __forceinline__ void adam_fold_body(const float *work, int nchunk, float *w, float *b, float *mw,
                                               float *vw, float *mb, float *vb, int co, int ci, uint16_t *packed,
                                               uint16_t *packed_flip, const float *hyper, float *gw, float *gb,
                                               int block) {
    bool ok;
    const float t = fold_output(work, nchunk, ci, co, true, ok, block);
    if (threadIdx.x >= 64 || !ok) return;
    const int nw = co * kTaps * ci, idx = block * 64 + threadIdx.x;
    if (idx < nw) {
        if (gw) gw[idx] = t;
    } else if (gb) {
        gb[idx - nw] = t;
    }
    adam_layer_param(idx, t, w, b, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper);
}

__global__ __launch_bounds__(64 * kFoldWaves) void adam_fold_kernel(const float *work, int nchunk, float *w, float *b,
                                                                    float *mw, float *vw, float *mb, float *vb,
                                                                    int co, int ci, uint16_t *packed,
                                                                    uint16_t *packed_flip, const float *hyper,
                                                                    float *gw, float *gb) {
    adam_fold_body(work, nchunk, w, b, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper, gw, gb, blockIdx.x);
}

// The same for up to LBM_CNN_MAX_LAYERS layers in one launch: layer l owns
// workgroups first[l] .. first[l + 1] - 1.
struct FoldLayers {
    lbm_cnn_layer layer[LBM_CNN_MAX_LAYERS];
    int first[LBM_CNN_MAX_LAYERS + 1];
    int nlayers, nchunk;
    const float *hyper;
};

__global__ __launch_bounds__(64 * kFoldWaves) void adam_fold_layers_kernel(const FoldLayers f) {
    const int b = blockIdx.x;
    int l = 0;
    while (l + 1 < f.nlayers && b >= f.first[l + 1]) ++l;
    const lbm_cnn_layer &L = f.layer[l];
    adam_fold_body(L.work, f.nchunk, L.w, L.b, L.mw, L.vw, L.mb, L.vb, L.co, L.ci, L.packed, L.packed_flip,
                   f.hyper, L.gw, L.gb, b - f.first[l]);
}

// Opens an optimizer step: hyper[0..3] = (lr, beta1, beta2, eps), hyper[4] += 1.
__global__ void adam_begin_kernel(float *hyper, float lr, float b1, float b2, float eps) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    hyper[0] = lr;
    hyper[1] = b1;
    hyper[2] = b2;
    hyper[3] = eps;
    hyper[4] = hyper[4] + 1.0f;
}

int32_t launched() { return hipGetLastError() == hipSuccess ? 0 : -3; }

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// The weight-gradient partials (the specialised kernel where it applies).
void launch_wgrad(const float *x, const float *gz, int n, int d, int h, int wd, int ci, int co, float *work,
                  int nchunk, hipStream_t st) {
    const dim3 grid(nchunk, pad16(kTaps * pad4(ci)) / 16, pad16(co) / 16);
    if (wd % 4 == 0 && pad4(ci) == 16)
        hipLaunchKernelGGL(conv_wgrad_x3, dim3(nchunk, kTaps / 3, pad16(co) / 16), dim3(256), 0, st, x, gz, n, d, h,
                           wd, ci, co, work);
    else if (wd % 4 == 0 && pad4(ci) == 4)
        hipLaunchKernelGGL(conv_wgrad_ci<4>, grid, dim3(256), 0, st, x, gz, n, d, h, wd, ci, co, work);
    else
        hipLaunchKernelGGL(conv_wgrad_kernel, grid, dim3(256), 0, st, x, gz, n, d, h, wd, ci, co, work);
}

}  // namespace

extern "C" {

int64_t lbm_cnn_packed_size(int32_t co, int32_t ci) {
    if (co < 1 || ci < 1) return -1;
    return (int64_t)pad16(co) * pad16(kTaps * pad4(ci));
}

int32_t lbm_cnn_pack_weights(const float *w, int32_t co, int32_t ci, int32_t flip, uint16_t *packed,
                             void *stream) {
    if (!w || !packed || co < 1 || ci < 1) return -1;
    const int rows16 = flip ? pad16(ci) : pad16(co);
    const int k16 = flip ? pad16(kTaps * pad4(co)) : pad16(kTaps * pad4(ci));
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for((int64_t)rows16 * k16, 256)), dim3(256), 0,
                       (hipStream_t)stream, w, co, ci, flip, packed, rows16, k16);
    return launched();
}

int32_t lbm_cnn_conv3d_forward(const float *x, int32_t n, int32_t d, int32_t h, int32_t wd, int32_t ci,
                               const uint16_t *packed, int32_t co, const float *bias, int32_t relu,
                               const float *mask, float *y, void *stream) {
    if (!x || !packed || !y || n < 1 || d < 1 || h < 1 || wd < 1 || ci < 1 || co < 1) return -1;
    if (((uintptr_t)x) % 16 || ((uintptr_t)packed) % 8) return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31)) return -1;
    const dim3 grid(blocks_for(nv, 64), pad16(co) / 16), grid8(blocks_for(nv, 128), pad16(co) / 16);
    if (pad4(ci) == 16)
        hipLaunchKernelGGL(conv_forward_ci<16>, grid8, dim3(512), 0, (hipStream_t)stream, x, n, d, h, wd, packed,
                           co, bias, relu, mask, y);
    else if (pad4(ci) == 4)
        hipLaunchKernelGGL(conv_forward_ci<4>, grid8, dim3(512), 0, (hipStream_t)stream, x, n, d, h, wd, packed,
                           co, bias, relu, mask, y);
    else
        hipLaunchKernelGGL(conv_forward_kernel, grid, dim3(256), 0, (hipStream_t)stream, x, n, d, h, wd, ci,
                           packed, co, bias, relu, mask, y);
    return launched();
}

int64_t lbm_cnn_wgrad_workspace(int32_t n, int32_t d, int32_t h, int32_t wd, int32_t ci, int32_t co) {
    if (n < 1 || d < 1 || h < 1 || wd < 1 || ci < 1 || co < 1) return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    const int64_t nchunk = (nv + kWgradVoxels - 1) / kWgradVoxels;
    return nchunk * pad16(co) * (pad16(kTaps * pad4(ci)) + 1) * (int64_t)sizeof(float);
}

int32_t lbm_cnn_conv3d_wgrad(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                             int32_t ci, int32_t co, float *work, float *gw, float *gb, void *stream) {
    if (!x || !gz || !work || !gw || n < 1 || d < 1 || h < 1 || wd < 1 || ci < 1 || co < 1) return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31)) return -1;
    const int nchunk = (int)((nv + kWgradVoxels - 1) / kWgradVoxels);
    hipStream_t st = (hipStream_t)stream;
    launch_wgrad(x, gz, n, d, h, wd, ci, co, work, nchunk, st);
    hipLaunchKernelGGL(grad_fold_kernel, dim3(blocks_for((int64_t)co * kTaps * ci + co, 64)), dim3(64 * kFoldWaves),
                       0, st, work, nchunk, ci, co, gw, gb);
    return launched();
}

int32_t lbm_cnn_conv3d_wgrad_partials(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                                      int32_t ci, int32_t co, float *work, void *stream) {
    if (!x || !gz || !work || n < 1 || d < 1 || h < 1 || wd < 1 || ci < 1 || co < 1) return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31)) return -1;
    const int nchunk = (int)((nv + kWgradVoxels - 1) / kWgradVoxels);
    launch_wgrad(x, gz, n, d, h, wd, ci, co, work, nchunk, (hipStream_t)stream);
    return launched();
}

int32_t lbm_cnn_backward_layer(const float *x, const float *gz, int32_t n, int32_t d, int32_t h, int32_t wd,
                               int32_t ci, int32_t co, float *work, const uint16_t *packed_flip, const float *mask,
                               float *gin, void *stream) {
    if (!x || !gz || !work || !packed_flip || !gin || n < 1 || d < 1 || h < 1 || wd < 1 || ci < 1 || co < 1)
        return -1;
    if (((uintptr_t)gz) % 16 || ((uintptr_t)packed_flip) % 8) return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31)) return -1;
    const int nchunk = (int)((nv + kWgradVoxels - 1) / kWgradVoxels);
    const int wi = pad4(ci), fi = pad4(co);
    // weight-gradient workgroups per (chunk, output tile): 16-column tiles, or
    // for 16 input channels groups of three taps
    const int nk = wi == 16 ? kTaps / 3 : pad16(kTaps * wi) / 16, nc = pad16(co) / 16;
    const int fx = (int)blocks_for(nv, 64), fy = pad16(ci) / 16;
    const int64_t total = (int64_t)nchunk * nk * nc + (int64_t)fx * fy;
    hipStream_t st = (hipStream_t)stream;
    if (wd % 4 == 0 && (wi == 4 || wi == 16) && (fi == 4 || fi == 16) && total < (int64_t(1) << 31)) {
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)total), dim3(256), 0, st, x, gz, n, d, h, wd, ci, co, work,
                               nchunk, nk, nc, packed_flip, mask, gin, fx);
        };
        if (wi == 16 && fi == 16) go(backward_layer_kernel<16, 16>);
        else if (wi == 16) go(backward_layer_kernel<16, 4>);
        else if (fi == 16) go(backward_layer_kernel<4, 16>);
        else go(backward_layer_kernel<4, 4>);
        return launched();
    }
    // other shapes: the two launches
    int32_t r = lbm_cnn_conv3d_wgrad_partials(x, gz, n, d, h, wd, ci, co, work, stream);
    if (r != 0) return r;
    return lbm_cnn_conv3d_forward(gz, n, d, h, wd, co, packed_flip, ci, nullptr, 0, mask, gin, stream);
}

int32_t lbm_cnn_relu_backward(const float *a, float *g, int64_t count, void *stream) {
    if (!a || !g || count < 0) return -1;
    if (count == 0) return 0;
    hipLaunchKernelGGL(relu_backward_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, (hipStream_t)stream, a,
                       g, count);
    return launched();
}

int32_t lbm_cnn_mse(const float *y, int32_t ystride, const float *target, int64_t count, float *g,
                    float *loss, void *stream) {
    if (!y || !target || !g || !loss || ystride < 1 || count < 1) return -1;
    const int nb = (int)std::min<int64_t>(kLossBlocks, (count + 255) / 256);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, (hipStream_t)stream, y, ystride, target, count, g, loss);
    hipLaunchKernelGGL(mse_fold_kernel, dim3(1), dim3(kLossBlocks), 0, (hipStream_t)stream, loss, nb, count);
    return launched();
}

int32_t lbm_cnn_adam(float *w, const float *g, float *m, float *v, int64_t count, float lr, float beta1,
                     float beta2, float eps, int32_t t, void *stream) {
    if (!w || !g || !m || !v || count < 0 || t < 1) return -1;
    if (count == 0) return 0;
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                       count, lr, beta1, beta2, eps, c1, c2);
    return launched();
}

int32_t lbm_cnn_adam_begin(float *hyper, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!hyper || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return -1;
    hipLaunchKernelGGL(adam_begin_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, hyper, lr, beta1, beta2, eps);
    return launched();
}

int32_t lbm_cnn_adam_layer(float *w, float *b, const float *gw, const float *gb, float *mw, float *vw, float *mb,
                           float *vb, int32_t co, int32_t ci, uint16_t *packed, uint16_t *packed_flip,
                           const float *hyper, void *stream) {
    if (!w || !b || !gw || !gb || !mw || !vw || !mb || !vb || !packed || !packed_flip || !hyper || co < 1 || ci < 1)
        return -1;
    if ((int64_t)co * kTaps * ci + co >= (int64_t(1) << 31)) return -1;
    const int64_t n = (int64_t)co * kTaps * ci + co;
    hipLaunchKernelGGL(adam_layer_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, (hipStream_t)stream, w, b, gw, gb,
                       mw, vw, mb, vb, co, ci, packed, packed_flip, hyper);
    return launched();
}

int32_t lbm_cnn_adam_layer_fold(float *w, float *b, const float *work, int32_t n, int32_t d, int32_t h, int32_t wd,
                                float *mw, float *vw, float *mb, float *vb, int32_t co, int32_t ci, uint16_t *packed,
                                uint16_t *packed_flip, const float *hyper, float *gw, float *gb, void *stream) {
    if (!w || !b || !work || !mw || !vw || !mb || !vb || !packed || !packed_flip || !hyper || co < 1 || ci < 1 ||
        n < 1 || d < 1 || h < 1 || wd < 1)
        return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31) || (int64_t)co * kTaps * ci + co >= (int64_t(1) << 31)) return -1;
    const int nchunk = (int)((nv + kWgradVoxels - 1) / kWgradVoxels);
    hipLaunchKernelGGL(adam_fold_kernel, dim3(blocks_for((int64_t)co * kTaps * ci + co, 64)), dim3(64 * kFoldWaves),
                       0, (hipStream_t)stream, work, nchunk, w, b, mw, vw, mb, vb, co, ci, packed, packed_flip, hyper,
                       gw, gb);
    return launched();
}

int32_t lbm_cnn_adam_layers_fold(int32_t nlayers, const lbm_cnn_layer *layers, int32_t n, int32_t d, int32_t h,
                                 int32_t wd, const float *hyper, void *stream) {
    if (!layers || !hyper || nlayers < 1 || nlayers > LBM_CNN_MAX_LAYERS || n < 1 || d < 1 || h < 1 || wd < 1)
        return -1;
    const int64_t nv = (int64_t)n * d * h * wd;
    if (nv >= (int64_t(1) << 31)) return -1;
    FoldLayers f{};
    f.nlayers = nlayers;
    f.nchunk = (int)((nv + kWgradVoxels - 1) / kWgradVoxels);
    f.hyper = hyper;
    int64_t first = 0;
    for (int l = 0; l < nlayers; ++l) {
        const lbm_cnn_layer &L = layers[l];
        if (!L.w || !L.b || !L.work || !L.mw || !L.vw || !L.mb || !L.vb || !L.packed || !L.packed_flip ||
            L.co < 1 || L.ci < 1)
            return -1;
        f.layer[l] = L;
        f.first[l] = (int)first;
        first += blocks_for((int64_t)L.co * kTaps * L.ci + L.co, 64);
        if (first >= (int64_t(1) << 31)) return -1;
    }
    f.first[nlayers] = (int)first;
    hipLaunchKernelGGL(adam_fold_layers_kernel, dim3((unsigned)first), dim3(64 * kFoldWaves), 0,
                       (hipStream_t)stream, f);
    return launched();
}

int32_t lbm_cnn_adam_dev(float *w, const float *g, float *m, float *v, int64_t count, const float *hyper,
                         void *stream) {
    if (!w || !g || !m || !v || !hyper || count < 0) return -1;
    if (count == 0) return 0;
    hipLaunchKernelGGL(adam_dev_kernel, dim3(blocks_for(count, 256)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                       count, hyper);
    return launched();
}

}  // extern "C"
