// Control-variate network: parameter layout and host entry points.
#pragma once

#include <cstdint>

#include "pdd.h"

struct pdd_ctx;

namespace pdd {

constexpr int MLP_W = PDD_MLP_WIDTH;            // 64
constexpr int MLP_PARAMS = PDD_MLP_PARAMS;      // 4417
// offsets of W1[64][2], b1, W2[64][64] (out, in), b2, w3, b3 in the parameter vector
constexpr int OW1 = 0, OB1 = 128, OW2 = 192, OB2 = 4288, OW3 = 4352, OB3 = 4416;
static_assert(OB3 + 1 == MLP_PARAMS, "parameter layout");

pdd_status run_mlp_init(pdd_ctx* ctx, float* params, uint64_t seed);
pdd_status run_mlp_eval(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* v, float* g);
pdd_status run_mlp_grad_bf16(pdd_ctx* ctx, const float* params, int64_t n, const float* xy, float* g);
pdd_status run_mlp_bake(pdd_ctx* ctx, const float* params, const pdd_partition& part, int32_t lut_n, float* out);
pdd_status run_mlp_train(pdd_ctx* ctx, float* params, float* m, float* s, int64_t n_points, const float* xy,
                         const float* target, const int32_t* order, int64_t n_order, int32_t batch, int32_t steps,
                         int32_t step0, float lr, float* losses, float* grad_out);

}  // namespace pdd
