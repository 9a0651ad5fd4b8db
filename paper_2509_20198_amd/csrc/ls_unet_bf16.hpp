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

// Backward helpers (BF16 operands, FP32 results).
size_t ls_bf16_dpacked_offset(int layer);
size_t ls_bf16_dpacked_total();
int ls_bf16_prep_dgrad_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st);
int ls_bf16_mask_round(const float* g, const uint16_t* act, uint16_t* out, int64_t n, hipStream_t st);
int ls_bf16_embed8(const float* g, uint16_t* out, int64_t npix, hipStream_t st);
int ls_bf16_dgrad(const ConvSrc& s, int B, int H, int layer, const uint16_t* dpacked, float* out, hipStream_t st);
