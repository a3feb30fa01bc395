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

}  // namespace supa
