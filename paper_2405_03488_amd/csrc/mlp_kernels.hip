// Learned-proposal MLP on MFMA (gfx950): s = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,
// 16 -> 64 -> 64 -> 1, BF16 operands, FP32 accumulation, FP32 master weights.
//
// A wave handles rows in tiles of 16 with v_mfma_f32_16x16x16_bf16.  Operand
// layout of one 16x16x16 product (lane l, element i = 0..3):
//   A[m][k] : m = l % 16, k = 4 (l / 16) + i
//   B[k][n] : n = l % 16, k = 4 (l / 16) + i
//   D[m][n] : n = l % 16, m = 4 (l / 16) + i
// so an activation tile held in D layout is, unchanged, the A operand of its
// transpose and the B operand of itself: the weight gradients H1^T dZ2 and
// X^T dZ1 need no data movement; H1 and dZ2 go through LDS once per tile to
// become A operands of the next product.
// Loss = mean over the minibatch of (s - y)^2 / 2.  The four waves of a block
// add their gradients into one LDS copy in wave order, the block writes it as
// its partial, and the partials are added in block order: the result does not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include "sgpm_internal.h"

namespace sgpm {

namespace {

constexpr int NIN = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH,
              OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_round(float f) {
    return __uint_as_float(((uint32_t)(uint16_t)bf16_bits(f)) << 16);
}

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

__device__ __forceinline__ float group16_sum(float x) {  // over lanes with the same l / 16
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ float across_groups(float x) {  // over the four groups, same l % 16
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

// B fragment of a row-major [K x 64] matrix W, K block kb, column block nb
__device__ __forceinline__ s4 frag_b(const float* W, int kb, int nb, int lane) {
    const int k0 = 16 * kb + 4 * (lane >> 4), n = 16 * nb + (lane & 15);
    s4 r;
    r.x = bf16_bits(W[(k0 + 0) * NH + n]);
    r.y = bf16_bits(W[(k0 + 1) * NH + n]);
    r.z = bf16_bits(W[(k0 + 2) * NH + n]);
    r.w = bf16_bits(W[(k0 + 3) * NH + n]);
    return r;
}
// B fragment of W2^T: B[kk][m] = W2[m][kk], kk block kb, m block mb
__device__ __forceinline__ s4 frag_bt(const float* W2, int kb, int mb, int lane) {
    const int kk0 = 16 * kb + 4 * (lane >> 4), m = 16 * mb + (lane & 15);
    s4 r;
    r.x = bf16_bits(W2[m * NH + kk0 + 0]);
    r.y = bf16_bits(W2[m * NH + kk0 + 1]);
    r.z = bf16_bits(W2[m * NH + kk0 + 2]);
    r.w = bf16_bits(W2[m * NH + kk0 + 3]);
    return r;
}

// Forward (and optionally backward) over rows [row0, row0 + nrows) of X, one
// wave.  With BWD every wave of the block must call it (nrows may be 0): the
// waves add their gradients into gacc (NPARAM floats of LDS) in wave order.
template <bool BWD>
__device__ __forceinline__ void mlp_wave(const float* __restrict__ P, const float* __restrict__ X, const float* __restrict__ y,
                         int64_t row0, int nrows, float inv_batch, float* __restrict__ s_out, float* gacc,
                         float* lds /* 16 x 64 floats */) {
    const int lane = (int)(threadIdx.x & 63), col = lane & 15, grp = lane >> 4;
    const float* W1 = P + OFF_W1;
    const float* W2 = P + OFF_W2;
    f4 gW1[4], gW2[4][4];
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.f;
    if (BWD) {
        for (int a = 0; a < 4; ++a) {
            gW1[a] = f4{0, 0, 0, 0};
            for (int b = 0; b < 4; ++b) gW2[a][b] = f4{0, 0, 0, 0};
        }
    }
    for (int t0 = 0; t0 < nrows; t0 += 16) {
        const int64_t r0 = row0 + t0;
        const int valid = min(16, nrows - t0);
        // A fragment of X: row l % 16, k = 4 grp + i (rows beyond the tile read as zero)
        s4 ax;
        {
            const bool ok = (lane & 15) < valid;
            const float* xr = X + (r0 + (lane & 15)) * NIN + 4 * grp;
            ax.x = bf16_bits(ok ? xr[0] : 0.f);
            ax.y = bf16_bits(ok ? xr[1] : 0.f);
            ax.z = bf16_bits(ok ? xr[2] : 0.f);
            ax.w = bf16_bits(ok ? xr[3] : 0.f);
        }
        // layer 1 (D layout: row 4 grp + i, column 16 nb + col)
        f4 z1[4], h1[4];
        for (int nb = 0; nb < 4; ++nb) {
            z1[nb] = mfma(ax, frag_b(W1, 0, nb, lane), f4{0, 0, 0, 0});
            const float bb = P[OFF_B1 + 16 * nb + col];
            for (int i = 0; i < 4; ++i) {
                z1[nb][i] += bb;
                h1[nb][i] = bf16_round(z1[nb][i] > 0.f ? z1[nb][i] : 0.f);
            }
        }
        // H1 to A layout through LDS
        for (int nb = 0; nb < 4; ++nb)
            for (int i = 0; i < 4; ++i) lds[(4 * grp + i) * NH + 16 * nb + col] = h1[nb][i];
        __builtin_amdgcn_wave_barrier();
        s4 ah[4];
        for (int kb = 0; kb < 4; ++kb) {
            const float* hr = lds + (lane & 15) * NH + 16 * kb + 4 * grp;
            ah[kb] = s4{bf16_bits(hr[0]), bf16_bits(hr[1]), bf16_bits(hr[2]), bf16_bits(hr[3])};
        }
        __builtin_amdgcn_wave_barrier();
        // layer 2
        f4 z2[4];
        float sp[4] = {0, 0, 0, 0};  // partial s for rows 4 grp + i
        for (int nb = 0; nb < 4; ++nb) {
            f4 acc = f4{0, 0, 0, 0};
            for (int kb = 0; kb < 4; ++kb) acc = mfma(ah[kb], frag_b(W2, kb, nb, lane), acc);
            const float bb = P[OFF_B2 + 16 * nb + col];
            const float w3 = bf16_round(P[OFF_W3 + 16 * nb + col]);
            for (int i = 0; i < 4; ++i) {
                acc[i] += bb;
                const float h2 = acc[i] > 0.f ? acc[i] : 0.f;
                sp[i] += h2 * w3;
            }
            z2[nb] = acc;
        }
        float s[4];
        for (int i = 0; i < 4; ++i) s[i] = group16_sum(sp[i]) + P[OFF_B3];
        if (s_out && col == 0)
            for (int i = 0; i < 4; ++i)
                if (4 * grp + i < valid) s_out[r0 + 4 * grp + i] = s[i];
        if (!BWD) continue;
        // ---- backward
        float ds[4];
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * grp + i;
            ds[i] = r < valid ? (s[i] - y[r0 + r]) * inv_batch : 0.f;
            if (col == 0) gb3 += ds[i];
        }
        f4 dz2[4];
        for (int nb = 0; nb < 4; ++nb) {
            const float w3 = bf16_round(P[OFF_W3 + 16 * nb + col]);
            for (int i = 0; i < 4; ++i) {
                const float h2 = z2[nb][i] > 0.f ? z2[nb][i] : 0.f;
                gw3[nb] += ds[i] * h2;
                dz2[nb][i] = z2[nb][i] > 0.f ? ds[i] * w3 : 0.f;
                gb2[nb] += dz2[nb][i];
            }
        }
        // gW2 += H1^T dZ2: H1 (D layout) is the A operand of H1^T, dZ2 (D layout) the B operand
        s4 bdz[4];
        for (int nb = 0; nb < 4; ++nb)
            bdz[nb] = s4{bf16_bits(dz2[nb][0]), bf16_bits(dz2[nb][1]), bf16_bits(dz2[nb][2]), bf16_bits(dz2[nb][3])};
        for (int mb = 0; mb < 4; ++mb) {
            const s4 ah1t = s4{bf16_bits(h1[mb][0]), bf16_bits(h1[mb][1]), bf16_bits(h1[mb][2]), bf16_bits(h1[mb][3])};
            for (int nb = 0; nb < 4; ++nb) gW2[mb][nb] = mfma(ah1t, bdz[nb], gW2[mb][nb]);
        }
        // dH1 = dZ2 W2^T: dZ2 to A layout through LDS
        for (int nb = 0; nb < 4; ++nb)
            for (int i = 0; i < 4; ++i) lds[(4 * grp + i) * NH + 16 * nb + col] = dz2[nb][i];
        __builtin_amdgcn_wave_barrier();
        s4 adz[4];
        for (int kb = 0; kb < 4; ++kb) {
            const float* dr = lds + (lane & 15) * NH + 16 * kb + 4 * grp;
            adz[kb] = s4{bf16_bits(dr[0]), bf16_bits(dr[1]), bf16_bits(dr[2]), bf16_bits(dr[3])};
        }
        __builtin_amdgcn_wave_barrier();
        // X^T as an A operand: A[m = input][kk = row] = X[row = 4 grp + i][input = col]
        s4 axt;
        {
            float xv[4];
            for (int i = 0; i < 4; ++i) {
                const int r = 4 * grp + i;
                xv[i] = r < valid ? X[(r0 + r) * NIN + col] : 0.f;
            }
            axt = s4{bf16_bits(xv[0]), bf16_bits(xv[1]), bf16_bits(xv[2]), bf16_bits(xv[3])};
        }
        for (int mb = 0; mb < 4; ++mb) {
            f4 dh = f4{0, 0, 0, 0};
            for (int kb = 0; kb < 4; ++kb) dh = mfma(adz[kb], frag_bt(W2, kb, mb, lane), dh);
            f4 dz1;
            for (int i = 0; i < 4; ++i) {
                dz1[i] = z1[mb][i] > 0.f ? dh[i] : 0.f;
                gb1[mb] += dz1[i];
            }
            const s4 bdz1 = s4{bf16_bits(dz1[0]), bf16_bits(dz1[1]), bf16_bits(dz1[2]), bf16_bits(dz1[3])};
            gW1[mb] = mfma(axt, bdz1, gW1[mb]);
        }
    }
    if (!BWD) return;
    float gv1[4], gv2[4], gv3[4];
    for (int nb = 0; nb < 4; ++nb) {
        gv1[nb] = across_groups(gb1[nb]);
        gv2[nb] = across_groups(gb2[nb]);
        gv3[nb] = across_groups(gw3[nb]);
    }
    float g3 = gb3;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) g3 += __shfl_xor(g3, o);
    // this wave's gradient (D layouts -> parameter indices) into gacc, wave 0
    // storing and waves 1-3 adding, one wave per phase
    const int wid = (int)(threadIdx.x >> 6);
    for (int phase = 0; phase < 4; ++phase) {
        if (wid == phase) {
            auto put = [&](int idx, float v) { gacc[idx] = phase == 0 ? v : gacc[idx] + v; };
            for (int mb = 0; mb < 4; ++mb)
                for (int i = 0; i < 4; ++i) put(OFF_W1 + (4 * grp + i) * NH + 16 * mb + col, gW1[mb][i]);
            for (int mb = 0; mb < 4; ++mb)
                for (int nb = 0; nb < 4; ++nb)
                    for (int i = 0; i < 4; ++i) put(OFF_W2 + (16 * mb + 4 * grp + i) * NH + 16 * nb + col, gW2[mb][nb][i]);
            if (grp == 0)
                for (int nb = 0; nb < 4; ++nb) {
                    put(OFF_B1 + 16 * nb + col, gv1[nb]);
                    put(OFF_B2 + 16 * nb + col, gv2[nb]);
                    put(OFF_W3 + 16 * nb + col, gv3[nb]);
                }
            if (lane == 0) put(OFF_B3, g3);
        }
        __syncthreads();
    }
}

// rows split over waves: wave w takes rows [w * per, (w + 1) * per)
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                          int64_t N, int per_wave, float* __restrict__ s_out) {
    __shared__ float lds[4][16 * NH];
    const int w = (int)(threadIdx.x >> 6);
    const int64_t wave = (int64_t)blockIdx.x * 4 + w;
    const int64_t r0 = wave * per_wave;
    if (r0 >= N) return;
    const int nrows = (int)min((int64_t)per_wave, N - r0);
    mlp_wave<false>(P, X, nullptr, r0, nrows, 0.f, s_out, nullptr, lds[w]);
}

// one partial gradient per block: its four waves' rows [r0, r0 + per_wave)
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                       const float* __restrict__ y, int64_t N, int per_wave,
                                                       float inv_batch, float* __restrict__ gpart) {
    __shared__ float lds[4][16 * NH];
    __shared__ float gacc[NPARAM];
    const int w = (int)(threadIdx.x >> 6);
    const int64_t wave = (int64_t)blockIdx.x * 4 + w;
    const int64_t r0 = wave * per_wave;
    const int nrows = r0 < N ? (int)min((int64_t)per_wave, N - r0) : 0;
    mlp_wave<true>(P, X, y, r0, nrows, inv_batch, nullptr, gacc, lds[w]);
    float* gout = gpart + (int64_t)blockIdx.x * NPARAM;
    for (int i = (int)threadIdx.x; i < NPARAM; i += 256) gout[i] = gacc[i];
}

// grads = sum of the block partials in block order
__global__ void sum_partials_kernel(const float* __restrict__ gpart, int nparts, float* __restrict__ g) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= NPARAM) return;
    float a = 0.f;
    for (int w = 0; w < nparts; ++w) a += gpart[(int64_t)w * NPARAM + i];
    g[i] = a;
}

__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ gpart, int nparts, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= NPARAM) return;
    float g = 0.f;
    for (int w = 0; w < nparts; ++w) g += gpart[(int64_t)w * NPARAM + i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam over nsteps consecutive minibatches of B rows in one workgroup, for
// minibatches one gradient block covers (B <= 256): the weights stay in LDS
// between steps and the moments in registers (thread t owns parameters
// t + 256 k every step), so a step costs no launch and no global access but
// its rows.  The arithmetic is that of
// mlp_grad_kernel + adam_kernel step by step: the gradient rows split over the
// four waves as grad_rows_per_wave gives them, the bias corrections from the
// running products beta^t, carried in from the caller as pb1, pb2.
__global__ __launch_bounds__(256) void mlp_train_kernel(float* __restrict__ P, float* __restrict__ m,
                                                        float* __restrict__ v, const float* __restrict__ X,
                                                        const float* __restrict__ y, int64_t nsteps, int B,
                                                        int per_wave, float lr, float pb1, float pb2) {
    __shared__ float lds[4][16 * NH];
    __shared__ float gacc[NPARAM];
    __shared__ float Pl[NPARAM];
    constexpr int PPT = (NPARAM + 255) / 256;
    const int tid = (int)threadIdx.x, w = tid >> 6;
    float mr[PPT], vr[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = tid + 256 * k;
        mr[k] = i < NPARAM ? m[i] : 0.f;
        vr[k] = i < NPARAM ? v[i] : 0.f;
        if (i < NPARAM) Pl[i] = P[i];
    }
    __syncthreads();
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f, inv = 1.f / (float)B;
    const int64_t r0 = (int64_t)w * per_wave;
    const int nrows = r0 < B ? (int)min((int64_t)per_wave, (int64_t)B - r0) : 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        mlp_wave<true>(Pl, X + s * B * NIN, y + s * B, r0, nrows, inv, nullptr, gacc, lds[w]);
        pb1 *= b1;
        pb2 *= b2;
        const float c1 = 1.f - pb1, c2 = 1.f - pb2;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = tid + 256 * k;
            if (i < NPARAM) {
                const float g = gacc[i];
                mr[k] = b1 * mr[k] + (1.f - b1) * g;
                vr[k] = b2 * vr[k] + (1.f - b2) * g * g;
                Pl[i] -= lr * (mr[k] / c1) / (sqrtf(vr[k] / c2) + eps);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int i = tid + 256 * k;
        if (i < NPARAM) {
            P[i] = Pl[i];
            m[i] = mr[k];
            v[i] = vr[k];
        }
    }
}

}  // namespace

int mlp_nparams() { return NPARAM; }

// Gradient launches: up to 1024 blocks (4 per CU at this kernel's LDS use, on
// 256 CUs), each wave taking a run of rows that is a multiple of the 16-row tile.
int64_t mlp_grad_blocks(int64_t N) {
    const int64_t b = (N + 255) / 256;
    return b < 1 ? 1 : b > 1024 ? 1024 : b;
}
static int grad_rows_per_wave(int64_t N) {
    const int64_t waves = 4 * mlp_grad_blocks(N);
    const int64_t per = (N + waves - 1) / waves;
    return (int)((per + 15) / 16 * 16);
}

hipError_t mlp_forward(const float* P, const float* X, int64_t N, float* s_out, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const int per = 64;
    const int64_t waves = (N + per - 1) / per;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, st, P, X, N, per, s_out);
    return hipGetLastError();
}

// gradient of the mean loss over rows [0, N) into g (NPARAM floats); gpart holds
// mlp_grad_blocks(N) x NPARAM floats
hipError_t mlp_grad(const float* P, const float* X, const float* y, int64_t N, float* gpart, float* g,
                    hipStream_t st) {
    const unsigned blocks = (unsigned)mlp_grad_blocks(N);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(256), 0, st, P, X, y, N, grad_rows_per_wave(N),
                       1.f / (float)N, gpart);
    hipLaunchKernelGGL(sum_partials_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, gpart, (int)blocks, g);
    return hipGetLastError();
}

// Adam steps on nsteps consecutive minibatches of B rows (step s takes rows
// [s B, (s + 1) B) of X, y).  bpow = {0.9^t, 0.999^t} before the first step,
// host memory, advanced by nsteps.  One launch in all when a minibatch fits one
// gradient block, else a gradient and an update launch per step (gpart holds
// mlp_grad_blocks(B) x NPARAM floats).
hipError_t mlp_adam_steps(float* P, float* m, float* v, const float* X, const float* y, int64_t nsteps, int64_t B,
                          float lr, float* bpow, float* gpart, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f;
    const unsigned blocks = (unsigned)mlp_grad_blocks(B);
    if (nsteps <= 0) return hipSuccess;
    if (blocks == 1) {
        hipLaunchKernelGGL(mlp_train_kernel, dim3(1), dim3(256), 0, st, P, m, v, X, y, nsteps, (int)B,
                           grad_rows_per_wave(B), lr, bpow[0], bpow[1]);
        for (int64_t s = 0; s < nsteps; ++s) {
            bpow[0] *= b1;
            bpow[1] *= b2;
        }
        return hipGetLastError();
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(256), 0, st, P, X + s * B * NIN, y + s * B, B,
                           grad_rows_per_wave(B), 1.f / (float)B, gpart);
        bpow[0] *= b1;
        bpow[1] *= b2;
        const float c1 = 1.f - bpow[0], c2 = 1.f - bpow[1];
        hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, P, gpart, (int)blocks, m, v,
                           lr, b1, b2, 1e-8f, c1, c2);
    }
    return hipGetLastError();
}

}  // namespace sgpm
