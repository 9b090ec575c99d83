// Learned order predictor (filled in with the MLP kernels).
#include "plan_host.h"

sft_status sft_mlp_enqueue_orders(sft_plan_t plan, const signed char** orders) {
    (void)plan;
    *orders = nullptr;
    return SFT_E_INVALID;
}
