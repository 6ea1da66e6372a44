// Policy network on the inference path: stacked observations -> logits ->
// greedy actions, all on the device.
//
// What it computes (paper, Section 4, the "inference only" load condition:
// a policy DNN selects the actions and both emulation and inference run on
// the GPU).  The paper does not give its network; this is the convolutional
// trunk common to the A2C/DQN agents it builds on: conv 32 x 8x8 stride 4,
// conv 64 x 4x4 stride 2, conv 64 x 3x3 stride 1 (ReLU after each), a
// 3136 -> 512 layer (ReLU), and a 512 -> 19 head (18 action logits and a
// value).  Inputs are the u8 stack [4][84][84] scaled by 1/255.  Weights and
// hidden activations are bf16, products accumulate in fp32 on the matrix
// cores (v_mfma_f32_16x16x32_bf16), biases are fp32; the action is the first
// maximal logit.  The first layer feeds the pixel values themselves (integers
// 0..255, exact in bf16) and applies the 1/255 to its fp32 sums.
//
// Every layer is one implicit GEMM, computed transposed: the matrix cores'
// first operand is a 16-channel slice of the weights, the second 16 output
// positions (env, oy, ox) whose receptive fields are gathered straight from
// the input activation (no im2col buffer).  A lane then ends with 4
// consecutive channels of one position, which it stores as one 8-byte (bf16)
// or 16-byte (fp32 logits) write into the NHWC output.  Activations are NHWC,
// so 8 consecutive reduction indices are 8 consecutive input channels (one
// 16-byte load); the first layer reads the u8 NCHW stack and orders its
// reduction as (channel, ky, kx), so 8 consecutive indices are an 8-pixel
// run of one input row (two 4-byte loads).
//
// Weights arrive pre-arranged in operand order (see policy_swizzle_index):
// fragment (k-step s, channel tile j) is 64 x 16 contiguous bytes, lane l's
// 8 values at l * 16, so a wave reads it as one linear 1 KB access, from LDS
// for the three convolutions (whole layer staged once per block, at most
// 72 KB) and from L2 for the two dense layers.  Layer shapes are template
// constants: every gather offset folds at compile time.
#include "vcs_device.h"

namespace vcs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t f2bf(float f) {   // round to nearest even
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// One layer's shape and blocking.  H: input side, CIN: input channels,
// KW: kernel side, S: stride, OH: output side, N: outputs, NT: 16-channel
// tiles (N padded), NBW: channel tiles per wave (grid.y = NT / NBW), MR:
// 16-position tiles per wave, TPB: block tiles per block.
template <uint32_t H_, uint32_t CIN_, uint32_t KW_, uint32_t S_, uint32_t OH_, uint32_t N_, uint32_t NT_,
          uint32_t NBW_, uint32_t MR_, uint32_t TPB_, bool FIRST_, bool HEAD_, bool LDSW_>
struct Layer {
    static constexpr uint32_t H = H_, CIN = CIN_, KW = KW_, S = S_, OH = OH_, N = N_, NT = NT_, NBW = NBW_,
                              MR = MR_, TPB = TPB_;
    static constexpr bool FIRST = FIRST_, HEAD = HEAD_, LDSW = LDSW_;
    static constexpr uint32_t K = KW * KW * CIN, KS = K / 32, OHW = OH * OH, ROWS = 64 * MR;
    static_assert(K % 32 == 0 && (FIRST ? KW == 8 : CIN % 32 == 0), "reduction blocking");
    static_assert(NT % NBW == 0, "channel tiles per wave");
};

using L1 = Layer<84, 4, 8, 4, 20, 32, 2, 2, 4, 4, true, false, true>;
using L2 = Layer<20, 32, 4, 2, 9, 64, 4, 4, 4, 2, false, false, true>;
using L3 = Layer<9, 64, 3, 1, 7, 64, 4, 4, 2, 1, false, false, true>;
using L4 = Layer<7, 64, 7, 1, 1, 512, 32, 4, 1, 1, false, false, false>;
using L5 = Layer<1, 512, 1, 1, 1, 19, 2, 2, 1, 1, false, true, false>;

// the second MFMA operand for k-step s: 8 reduction indices of one position
template <class L, uint32_t s>
__device__ __forceinline__ bf16x8 gather(const void* in, uint64_t base, uint32_t q) {
    if constexpr (L::FIRST) {
        // k = s * 32 + 8 q = (channel * 8 + ky) * 8 + kx: channel s / 2, ky 4 (s & 1) + q, kx 0..7
        const uint8_t* src = static_cast<const uint8_t*>(in) + base + ((s / 2) * L::H + 4 * (s & 1)) * L::H + q * L::H;
        const uint32_t w0 = *reinterpret_cast<const uint32_t*>(src);
        const uint32_t w1 = *reinterpret_cast<const uint32_t*>(src + 4);
        bf16x8 a;
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] = (__bf16)(float)(((t < 4 ? w0 : w1) >> (8 * (t & 3))) & 0xFF);
        return a;
    } else {
        // k = s * 32 + 8 q = (ky * KW + kx) * CIN + channel
        constexpr uint32_t kk = s * 32 / L::CIN, c0 = s * 32 % L::CIN;
        constexpr uint32_t off = ((kk / L::KW) * L::H + kk % L::KW) * L::CIN + c0;
        return *reinterpret_cast<const bf16x8*>(static_cast<const uint16_t*>(in) + base + off + 8 * q);
    }
}

template <class L, uint32_t s>
__device__ __forceinline__ void kstep(const void* in, const uint64_t (&base)[L::MR], uint32_t q,
                                      const bf16x8* wsrc, f32x4 (&acc)[L::MR][L::NBW]) {
    bf16x8 b[L::NBW], a[L::MR];
#pragma unroll
    for (uint32_t j = 0; j < L::NBW; ++j) b[j] = wsrc[(s * L::NT + j) * 64];
#pragma unroll
    for (uint32_t r = 0; r < L::MR; ++r) a[r] = gather<L, s>(in, base[r], q);
#pragma unroll
    for (uint32_t r = 0; r < L::MR; ++r)
#pragma unroll
        for (uint32_t j = 0; j < L::NBW; ++j)
            acc[r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[r], acc[r][j], 0, 0, 0);
}

template <class L, uint32_t... S>
__device__ __forceinline__ void ksteps(const void* in, const uint64_t (&base)[L::MR], uint32_t q, const bf16x8* wsrc,
                                       f32x4 (&acc)[L::MR][L::NBW], std::integer_sequence<uint32_t, S...>) {
    (kstep<L, S>(in, base, q, wsrc, acc), ...);
}

template <class L>
__global__ void __launch_bounds__(256) k_policy_layer(PolicyLayerArgs A) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4, p = lane & 15;
    const uint32_t jt0 = blockIdx.y * L::NBW;
    __shared__ bf16x8 sw[L::LDSW ? L::KS * L::NT * 64 : 1];
    const bf16x8* wsrc;
    if constexpr (L::LDSW) {
        const bf16x8* g = reinterpret_cast<const bf16x8*>(A.w);
        for (uint32_t i = threadIdx.x; i < L::KS * L::NT * 64; i += 256) sw[i] = g[i];
        __syncthreads();
        wsrc = sw + jt0 * 64 + lane;
    } else {
        wsrc = reinterpret_cast<const bf16x8*>(A.w) + jt0 * 64 + lane;
    }
    // this lane's output channels: 4 q .. 4 q + 3 of each of its channel tiles
    f32x4 bias[L::NBW];
#pragma unroll
    for (uint32_t j = 0; j < L::NBW; ++j)
        bias[j] = *reinterpret_cast<const f32x4*>(A.bias + (jt0 + j) * 16 + 4 * q);

    for (uint32_t t = 0; t < L::TPB; ++t) {
        const uint32_t mbase = (blockIdx.x * L::TPB + t) * L::ROWS + wave * 16 * L::MR;
        if (mbase >= A.M) break;
        uint64_t base[L::MR];
#pragma unroll
        for (uint32_t r = 0; r < L::MR; ++r) {
            uint32_t row = mbase + r * 16 + p;
            row = row < A.M ? row : A.M - 1;               // rows past the end recompute the last one
            const uint32_t env = row / L::OHW, pix = row % L::OHW, oy = pix / L::OH, ox = pix % L::OH;
            if constexpr (L::FIRST)
                base[r] = ((uint64_t)env * L::CIN * L::H + oy * L::S) * L::H + ox * L::S;
            else
                base[r] = (((uint64_t)env * L::H + oy * L::S) * L::H + ox * L::S) * L::CIN;
        }
        f32x4 acc[L::MR][L::NBW];
#pragma unroll
        for (uint32_t r = 0; r < L::MR; ++r)
#pragma unroll
            for (uint32_t j = 0; j < L::NBW; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (L::KS <= 18) {
            ksteps<L>(A.in, base, q, wsrc, acc, std::make_integer_sequence<uint32_t, L::KS>{});
        } else {
            // the 3136-long reduction: 7 k-steps per pass over one kernel row (7 x 64 channels = 14 steps)
            static_assert(L::KS % 14 == 0, "dense layer blocking");
            for (uint32_t s0 = 0; s0 < L::KS; s0 += 14) {
                const uint64_t sh = (uint64_t)(s0 / 14) * L::H * L::CIN;   // next kernel row
                uint64_t b2[L::MR];
#pragma unroll
                for (uint32_t r = 0; r < L::MR; ++r) b2[r] = base[r] + sh;
                ksteps<L>(A.in, b2, q, wsrc + s0 * L::NT * 64, acc, std::make_integer_sequence<uint32_t, 14>{});
            }
        }
        // lane holds position p of each 16-row tile and channels 4 q .. 4 q + 3 of each channel tile
#pragma unroll
        for (uint32_t r = 0; r < L::MR; ++r) {
            const uint32_t m = mbase + r * 16 + p;
            if (m >= A.M) continue;
#pragma unroll
            for (uint32_t j = 0; j < L::NBW; ++j) {
                const uint32_t c0 = (jt0 + j) * 16 + 4 * q;
                f32x4 v = acc[r][j];
                if constexpr (L::FIRST) v = v * (1.0f / 255.0f);
                v = v + bias[j];
                if constexpr (L::HEAD) {
                    *reinterpret_cast<f32x4*>(static_cast<float*>(A.out) + (size_t)m * 32 + c0) = v;
                } else {
                    const uint32_t lo = f2bf(v[0] > 0.f ? v[0] : 0.f) | (f2bf(v[1] > 0.f ? v[1] : 0.f) << 16);
                    const uint32_t hi = f2bf(v[2] > 0.f ? v[2] : 0.f) | (f2bf(v[3] > 0.f ? v[3] : 0.f) << 16);
                    *reinterpret_cast<uint2*>(static_cast<uint16_t*>(A.out) + (size_t)m * L::N + c0) = uint2{lo, hi};
                }
            }
        }
    }
}

template <class L>
static void launch_layer(const PolicyLayerArgs& a, hipStream_t s) {
    const uint32_t per_block = L::ROWS * L::TPB;
    const dim3 grid((a.M + per_block - 1) / per_block, L::NT / L::NBW);
    hipLaunchKernelGGL(k_policy_layer<L>, grid, dim3(256), 0, s, a);
}

// first maximal logit among the 18 actions; one thread per env
__global__ void k_argmax(const float* logits, uint32_t n, uint8_t* actions) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* l = logits + (size_t)i * 32;
    uint32_t best = 0;
    float bv = l[0];
    for (uint32_t a = 1; a < 18; ++a)
        if (l[a] > bv) {
            bv = l[a];
            best = a;
        }
    actions[i] = (uint8_t)best;
}

void launch_policy_layer(int layer, const PolicyLayerArgs& a, hipStream_t s) {
    switch (layer) {
        case 0: launch_layer<L1>(a, s); break;
        case 1: launch_layer<L2>(a, s); break;
        case 2: launch_layer<L3>(a, s); break;
        case 3: launch_layer<L4>(a, s); break;
        default: launch_layer<L5>(a, s); break;
    }
}

void launch_argmax(const float* logits, uint32_t n, uint8_t* actions, hipStream_t s) {
    hipLaunchKernelGGL(k_argmax, dim3((n + 255) / 256), dim3(256), 0, s, logits, n, actions);
}

}  // namespace vcs
