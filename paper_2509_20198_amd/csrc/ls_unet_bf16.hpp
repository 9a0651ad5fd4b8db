// BF16 (matrix-core) path of the refinement network.
#pragma once

#include "ls_common.hpp"
#include "ls_unet.hpp"

// Packed BF16 weights: per layer [Npad][Kpad], Npad = cout rounded up to 16,
// Kpad = 9*cin rounded up to 32, k = tap*cin + ci, zero padding.
size_t ls_bf16_packed_offset(int layer);
size_t ls_bf16_packed_total();
int ls_bf16_kpad(int layer);

int ls_bf16_prep_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st);
int ls_bf16_forward(const float* w, const uint16_t* packed, const float* x, int B, const LsGridInfo& gi,
                    uint16_t* acts, float* head, hipStream_t st);
int ls_pack_bf16(const float* w, uint16_t* out, int64_t n, hipStream_t st);
