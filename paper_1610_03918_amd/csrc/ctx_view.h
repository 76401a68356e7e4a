// Internal bridge between the two host runtimes of the library: what the
// learned start (unet_runtime.cpp) needs to see of a simulation context
// (pic_runtime.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

struct PicCtxView {
    const double *phi;          // current potential (the last solution on free nodes)
    const double *phi_prev;     // the solution before it, or null when the context has none
    const double *b;            // assembled right-hand side
    const uint8_t *node_cond;   // node map (0 free)
    int NX, NY, px, py;
    hipStream_t stream;         // the context's stream
};

// View of instance i of ctx; PIC_ERR_STATE / PIC_ERR_ARG on a bad context or instance.
__attribute__((visibility("hidden"))) pic_status pic_ctx_view(pic_ctx *ctx, int i, PicCtxView *out);
