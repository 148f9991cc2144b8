// Flow entries used by the integration loop.
//  flow_apply: transform n points of a [ndim][ld] FP32 array in place
//    (density direction, or sampling direction when inverse is set) and
//    write log q of each point.
//  flow_step: one training step on n points of a [ndim][ld] array with
//    per-point weights w (the weighted log-likelihood gradient,
//    -sum w grad log q / sum w) followed by Adam with rate lr; the loss value
//    goes to loss_dev (device).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/mf_flow.h"

namespace mf {
mf_status flow_apply(mf_flow* f, float* y, int64_t n, int64_t ld, float* logq, bool inverse, hipStream_t s);
mf_status flow_step(mf_flow* f, const float* y, int64_t ld, const float* w, int64_t n, float* loss_dev, double lr,
                    hipStream_t s);
}
