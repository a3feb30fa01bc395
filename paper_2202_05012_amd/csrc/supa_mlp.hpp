// supa_mlp.hpp -- arguments of the surrogate's matrix product kernels
// (supa_mlp.hip), shared with their C ABI (supa_surrogate_api.hip).
#pragma once
#include <stdint.h>

namespace supa {

// Arguments of the surrogate's matrix product (supa_mlp.hip).
struct GemmArgs {
    int M, N, K;
    const uint16_t *A;   // TA == 0: [M][lda] (row-major M x K); TA == 1: [K][lda] (K x M)
    const uint16_t *B;   // TB == 0: [K][ldb] (K x N);           TB == 1: [N][ldb] (N x K)
    int lda, ldb;
    const float *bias;   // [N] or null
    void *C;             // float [M][ldc] (EPI_F32, EPI_BIAS_F32) or bf16 [M][ldc]
    int ldc;
    uint16_t *pre;       // EPI_BIAS_GELU: pre-activation out; EPI_GELU_GRAD: in (bf16 [M][ldc])
    int k_chunk;         // > 0: block z covers K range [z k_chunk, (z+1) k_chunk) and writes
                         //   its partial product at C + z M ldc (EPI_F32); 0: all of K
    int split;           // EPI_GATE: columns from split on are log-variances
    float s_clamp;       // EPI_GATE: log-variance clamp
    const float *e0;     // EPI_GATE with counts: per row; a mean column counts as occupied when
    float cnt_scale;     //   mu > cnt_scale / e0[row] (null e0: no counts)
};

// Arguments of the fused forward pass (mlp_fused_kernel): an MLP of
// n_hidden GELU layers 256 wide on k_in inputs, then either the last hidden
// activations (n_out == 0) or a final linear layer of n_out outputs.
constexpr int MLP_FUSED_MAX_HIDDEN = 8;
struct MlpFusedArgs {
    int B, k_in, n_hidden, n_out;
    const uint16_t *x;   // bf16 [B][ldx], k_in columns
    int ldx;
    // layer l's weights transposed, bf16 [out][in]: in = k_in for l = 0, else
    // 256 with the input index permuted (the order the previous layer's
    // products leave the activations in registers)
    const uint16_t *wt[MLP_FUSED_MAX_HIDDEN + 1];
    const float *bias[MLP_FUSED_MAX_HIDDEN + 1];
    float *out;          // n_out > 0: float [B][ldo]
    int ldo;
    uint16_t *h;         // n_out == 0: bf16 [B][ldh], the last hidden activations
    int ldh;
};

}  // namespace supa
