// rt_mlp.h -- neural CO layer kernels (internal).
#pragma once
#include "../../include/rtcube.h"
#include "rt_kernels.h"

namespace rt {

// Prepared network: per hidden layer l the weights in the kernel's element
// type, row-major [128][K_l] (W) and transposed [K_l][128] (WT), float
// biases; the output layer in float; offsets of each layer in the flat
// float32 layout; the 16 Fourier frequencies.
struct MlpDev {
    const void *W[4];
    const void *WT[4];
    const float *b[4];
    const float *W5, *b5;
    int off[5];
    float freq[16];
    // BF16 only: the hidden layers as the A operand of the transposed product
    // (output neurons as rows), rows padded for LDS, input order of layers
    // 1..3 permuted to the accumulator layout of the layer before
    const void *Wr;
    // BF16 only: layers 1..3 transposed for the backward pass, [in][out slot]
    // with the output order permuted like the accumulator packing
    const void *WrT;
};

size_t mlp_prep_bytes(int precision);
hipError_t mlp_prepare(const float *flat, int precision, void *buf, MlpDev *w, hipStream_t st);
hipError_t mlp_forward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M, float4 *out,
                       hipStream_t st);
// list: device scratch of mlp_backward_list_bytes(M) (the BF16 backward's
// list of the passes with any dL/do != 0, and their flags)
size_t mlp_backward_list_bytes(size_t M);
hipError_t mlp_backward(const Geometry &g, const Shade &s, const MlpDev &w, int precision, size_t M,
                        const float4 *dO, uint32_t *list, float *dW, hipStream_t st);

} // namespace rt
