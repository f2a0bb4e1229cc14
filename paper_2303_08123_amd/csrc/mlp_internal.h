// Library-internal interface of the surrogate MLP: GEMM descriptor, views of
// the net and work buffers, and the passes built from the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gga {

enum : int { MLP_FWD = 0, MLP_BWD = 1, MLP_PLAIN = 2, MLP_INFER = 3, MLP_OUT = 4 };
constexpr int MLP_IN = 128, MLP_HID = 512, MLP_FRAC = 40;
constexpr long MLP_PARAMS = (long)MLP_IN * MLP_HID + MLP_HID + 2L * ((long)MLP_HID * MLP_HID + MLP_HID) + MLP_HID + 1;

struct MlpGemm {
    int M, N, K;
    const __bf16* A;
    long sa_m, sa_k;
    const __bf16* B;
    long sb_k, sb_n;
    const float* bias;
    int mode;
    float* Z;
    long ldz;
    __bf16* H;
    long ldh;
    float* C;
    long ldc;
    const float* w4;             // MLP_OUT: output weights; C receives partial dot products
};

// Views into a net buffer (see mlp_net()).
struct MlpNet {
    float* norm;                 // [2]: mu, sigma of the training targets
    int32_t* step;               // Adam step count (after norm in the same block)
    float *p, *m, *v, *g;        // [MLP_PARAMS] each
    float* Wf[3];                // fp32 master weights of the MFMA layers (views into p)
    const float* b[3];
    float *w4, *b4;
    float *gW[3], *gb[3], *gw4, *gb4;
    __bf16 *W[3], *WT[3];        // bf16 copies, [K][N] and [N][K]
};
constexpr int MLP_RED_CHUNKS = 64;   // row chunks of the batch reductions (bias gradients)
struct MlpWork {
    __bf16* X;
    float* Z[3];
    __bf16* H[3];
    float *y, *dy;
    __bf16* dZ[2];
    float* part;                 // [MLP_RED_CHUNKS][MLP_HID + 1] partial column sums
};
size_t mlp_net_bytes();
MlpNet mlp_net(void* base);
size_t mlp_work_bytes(int B);
void mlp_work_offsets(int B, size_t (&off)[12]);
MlpWork mlp_work(void* base, int B);

hipError_t launch_gemm(const MlpGemm& g, hipStream_t s);
hipError_t mlp_forward(const MlpNet& net, const float* dose, const int32_t* gap, const int32_t* nfrac, int B,
                       int K, const MlpWork& w, float* pred, bool predict, hipStream_t s);
hipError_t mlp_backward(const MlpNet& net, int B, const float* target, const MlpWork& w, float* loss,
                        hipStream_t s);
hipError_t mlp_adam_refresh(const MlpNet& net, int step, float lr, hipStream_t s);
hipError_t mlp_refresh_layer(const MlpNet& net, int l, hipStream_t s);
hipError_t mlp_init(const MlpNet& net, uint64_t seed, hipStream_t s);
hipError_t mlp_set_norm(const MlpNet& net, const float* t, int n, hipStream_t s);

}  // namespace gga
