// mlp_device.h -- the bfloat16 MFMA multilayer perceptron u_theta shared by
// the learned-proposal kernels: in -> 64 (ReLU) -> 64 (ReLU) -> out with FP32
// master parameters W1[64][in], b1[64], W2[64][64], b2[64], W3[out][64],
// b3[out], rounded to bfloat16 (nearest even) when loaded.
//
// MFMA mapping (v_mfma_f32_16x16x32_bf16).  A tile is 16 rows (grid nodes or
// training rows).  Every layer is computed transposed, H^T = W . X^T: the
// weights are the A operand (row = output unit; lane 16 g + row holds the 8
// K slots 8 g .. 8 g + 7), the activations the B operand (column = row of the
// tile).  The FP32 result of a layer -- lane 16 g + c holds units 4 g + r
// (r < 4) of every 16-unit block for tile row c -- is the B operand of the
// next layer as it stands once the next layer's weights use the matching K
// order: slot j of K-block kb in lane group g is hidden unit
// 16 (2 kb + j / 4) + 4 g + j % 4.  Layer 1 takes the inputs in slots
// 0 .. in-1, a constant 1 in slot `in` (whose weight column is b1) and zeros
// up to 32; layer 3 pads the outputs to 16 rows.  14 MFMAs per tile.
#pragma once

#include "pf_internal.h"

namespace pfk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = MLP_HIDDEN;
// inputs of the FH-N proposal: v patch (9), w patch (9), residual of the
// nearest observation, tau, the offsets of that observation (2)
constexpr int LEARNED_FEATURES = 22;

struct MlpRegs {
  bf16x8 a1[4];     // layer 1, one per block of 16 hidden units
  bf16x8 a2[4][2];  // layer 2 [output block][K block]
  bf16x8 a3[2];     // layer 3 [K block]
  f32x4 b2[4];      // bias of layer 2 in the accumulator layout
  f32x4 b3;         // bias of layer 3 in the accumulator layout
};

__device__ __forceinline__ int hid_slot(int kb, int g, int j) {
  return 16 * (2 * kb + (j >> 2)) + 4 * g + (j & 3);
}
__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }

__device__ inline void mlp_load(const float *__restrict__ p, int in_dim, int out_dim, MlpRegs &w) {
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
  const float *W1 = p, *b1 = W1 + HID * in_dim, *W2 = b1 + HID, *b2 = W2 + HID * HID;
  const float *W3 = b2 + HID, *b3 = W3 + out_dim * HID;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int u = 16 * b + c;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * g + j;
      const float v = k < in_dim ? W1[u * in_dim + k] : (k == in_dim ? b1[u] : 0.f);
      w.a1[b][j] = (__bf16)v;
    }
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob)
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) w.a2[ob][kb][j] = (__bf16)W2[(16 * ob + c) * HID + hid_slot(kb, g, j)];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      w.a3[kb][j] = (__bf16)(c < out_dim ? W3[c * HID + hid_slot(kb, g, j)] : 0.f);
#pragma unroll
  for (int ob = 0; ob < 4; ++ob)
#pragma unroll
    for (int r = 0; r < 4; ++r) w.b2[ob][r] = bf16r(b2[16 * ob + 4 * g + r]);
#pragma unroll
  for (int r = 0; r < 4; ++r) w.b3[r] = (4 * g + r) < out_dim ? bf16r(b3[4 * g + r]) : 0.f;
}

// ReLU as one integer max on the bit pattern: a float with the sign bit set
// (negative, or -0) is a negative int32 and becomes +0; others pass.
__device__ __forceinline__ float relu(float x) {
  return __int_as_float(max(__float_as_int(x), 0));
}

// ReLU, rounded to bfloat16, in the B-operand order of the next layer
__device__ __forceinline__ bf16x8 relu_pack(const f32x4 &lo, const f32x4 &hi) {
  bf16x8 o;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    o[r] = (__bf16)relu(lo[r]);
    o[4 + r] = (__bf16)relu(hi[r]);
  }
  return o;
}

// u_theta of the 16 tile rows whose features this lane holds in F (slots
// 8 g .. 8 g + 7 of row c).  Lane c of group 0 receives outputs 0..3 of row c.
__device__ __forceinline__ f32x4 mlp_tile(const MlpRegs &w, const bf16x8 &F) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  f32x4 a1[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) a1[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a1[b], F, z, 0, 0, 0);
  const bf16x8 h1[2] = {relu_pack(a1[0], a1[1]), relu_pack(a1[2], a1[3])};
  f32x4 a2[4];
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    a2[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a2[ob][0], h1[0], w.b2[ob], 0, 0, 0);
    a2[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a2[ob][1], h1[1], a2[ob], 0, 0, 0);
  }
  const bf16x8 h2[2] = {relu_pack(a2[0], a2[1]), relu_pack(a2[2], a2[3])};
  f32x4 o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a3[0], h2[0], w.b3, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w.a3[1], h2[1], o, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// The same network on v_mfma_f32_32x32x16_bf16 (tiles of 32 rows), which
// issues at about twice the rate of the 16x16x32 form on gfx950.  Operands:
// A lane 32 h + i holds A[i][8 h .. 8 h + 7] of a 16-wide K block, B lane
// 32 h + c holds B[8 h .. 8 h + 7][c], and element r of the 16 accumulators
// of lane 32 h + c is C[8 (r / 4) + 4 h + r % 4][c].  With the next layer's K
// slot j of K-block kb in lane half h taken as hidden unit
// 32 (kb / 2) + 8 (2 (kb % 2) + j / 4) + 4 h + j % 4, the B operand of K-block
// kb is accumulator elements 8 (kb % 2) .. 8 (kb % 2) + 7 of 32-unit block
// kb / 2, i.e. a contiguous slice.  Inputs: slots 16 kb + 8 h + j of the
// lane, the constant 1 in slot `in` (bias of layer 1).  Layers 1 and 2 take
// 4 + 8 MFMAs per 32 rows.
//
// Layer 3 (at most 4 outputs) runs on v_mfma_f32_4x4x4bf16_1k, 16
// independent 4x4x4 blocks: block b = lane / 4 takes row i of A from lane
// 4 b + i, column j of B from lane 4 b + j, and returns D[i][j] in element i
// of lane 4 b + j.  With B column j = the 4 hidden values that lane 4 b + j
// holds in one register pair (its own node, its half's units) and A row i =
// W3[i] at those units, 8 instructions leave in lane 32 h + c the sums of
// outputs 0..3 of row c over half h's 32 hidden units; one lane-half swap
// and an add finish them.  (A 32x32x16 layer 3 padded to 32 output rows
// took 4 instructions of 32 matrix-pipe cycles each; the 8 small ones take
// about 7 each.)
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct Mlp32Regs {
  bf16x8 a1[2][2];  // layer 1 [32-unit block][K block]
  bf16x8 a2[2][4];  // layer 2 [32-unit block][K block]
  bf16x4 a3[8];     // layer 3 [K block][register pair]: W3[lane % 4] at its units
  f32x16 b2[2];     // bias of layer 2 in the accumulator layout
  f32x4 c3;         // layer 3 accumulator start: its bias on lanes of half 0
};

__device__ __forceinline__ int hid_slot32(int kb, int h, int j) {
  return 32 * (kb >> 1) + 8 * (2 * (kb & 1) + (j >> 2)) + 4 * h + (j & 3);
}

// Input slot k = 16 kb + 8 h + j of layer 1 carries input slot_in(k): an
// index below in_dim, SLOT_ONE (the constant 1, whose weight column is b1) or
// SLOT_ZERO.  The default order is the inputs, then the 1, then zeros.
constexpr int SLOT_ONE = -1, SLOT_ZERO = -2;
struct InputsInOrder {
  int in_dim;
  __device__ int operator()(int k) const { return k < in_dim ? k : (k == in_dim ? SLOT_ONE : SLOT_ZERO); }
};

template <class SlotIn>
__device__ inline void mlp32_load(const float *__restrict__ p, int in_dim, int out_dim,
                                  Mlp32Regs &w, SlotIn slot_in) {
  const int l = threadIdx.x & 63, c = l & 31, h = l >> 5;
  const float *W1 = p, *b1 = W1 + HID * in_dim, *W2 = b1 + HID, *b2 = W2 + HID * HID;
  const float *W3 = b2 + HID, *b3 = W3 + out_dim * HID;
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    const int u = 32 * ob + c;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int f = slot_in(16 * kb + 8 * h + j);
        const float v = f >= 0 ? W1[u * in_dim + f] : (f == SLOT_ONE ? b1[u] : 0.f);
        w.a1[ob][kb][j] = (__bf16)v;
      }
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
      for (int j = 0; j < 8; ++j) w.a2[ob][kb][j] = (__bf16)W2[u * HID + hid_slot32(kb, h, j)];
#pragma unroll
    for (int r = 0; r < 16; ++r) w.b2[ob][r] = bf16r(b2[32 * ob + 8 * (r >> 2) + 4 * h + (r & 3)]);
  }
  const int o3 = l & 3;  // output row this lane supplies to layer 3's A
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      w.a3[2 * kb + j / 4][j % 4] =
          (__bf16)(o3 < out_dim ? W3[o3 * HID + hid_slot32(kb, h, j)] : 0.f);
#pragma unroll
  for (int r = 0; r < 4; ++r) w.c3[r] = (h == 0 && r < out_dim) ? bf16r(b3[r]) : 0.f;
}

// ReLU after the rounding, two values per instruction: rounding to nearest
// even keeps the sign, so a bfloat16 with its sign bit set (negative, -0) is a
// negative int16 and a packed integer max with 0 gives +0, which is the
// rounding of ReLU's result; the others pass unchanged.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 relu_pack8(const f32x16 &a, int off) {
  u32x4 q;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const f32x2 f = {a[off + 2 * j], a[off + 2 * j + 1]};
    const s16x2 b = __builtin_bit_cast(s16x2, __builtin_convertvector(f, bf16x2));
    q[j] = __builtin_bit_cast(unsigned, __builtin_elementwise_max(b, (s16x2){0, 0}));
  }
  return __builtin_bit_cast(bf16x8, q);
}

__device__ __forceinline__ float swap_halves_add(float lo_src, float hi_src) {
  // lanes of half 0 get lo_src(l) + lo_src(l + 32), lanes of half 1
  // hi_src(l - 32) + hi_src(l)
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo_src), __float_as_uint(hi_src),
                                                  false, false);
  return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// u_theta of the 32 tile rows whose inputs this lane holds (F[kb] = slots
// 16 kb + 8 h .. + 7 of row c).  Lane 32 h + c receives output h of row c in
// element 0 and (NOUT = 4) output 2 + h in element 1, bias included.
template <int NOUT>
__device__ __forceinline__ f32x2 mlp32_tile(const Mlp32Regs &w, const bf16x8 F[2]) {
  f32x16 z;
#pragma unroll
  for (int r = 0; r < 16; ++r) z[r] = 0.f;
  f32x16 a1[2];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    a1[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a1[ob][0], F[0], z, 0, 0, 0);
    a1[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a1[ob][1], F[1], a1[ob], 0, 0, 0);
  }
  const bf16x8 h1[4] = {relu_pack8(a1[0], 0), relu_pack8(a1[0], 8), relu_pack8(a1[1], 0),
                        relu_pack8(a1[1], 8)};
  f32x16 a2[2];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    a2[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a2[ob][0], h1[0], w.b2[ob], 0, 0, 0);
#pragma unroll
    for (int kb = 1; kb < 4; ++kb)
      a2[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w.a2[ob][kb], h1[kb], a2[ob], 0, 0, 0);
  }
  const bf16x8 h2[4] = {relu_pack8(a2[0], 0), relu_pack8(a2[0], 8), relu_pack8(a2[1], 0),
                        relu_pack8(a2[1], 8)};
  // layer 3: 8 small-block MFMAs over this half's hidden units, then the
  // two halves' sums
  f32x4 o = w.c3;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    o = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(w.a3[2 * kb],
                                               __builtin_shufflevector(h2[kb], h2[kb], 0, 1, 2, 3),
                                               o, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(w.a3[2 * kb + 1],
                                               __builtin_shufflevector(h2[kb], h2[kb], 4, 5, 6, 7),
                                               o, 0, 0, 0);
  }
  f32x2 u;
  u[0] = swap_halves_add(o[0], o[1]);
  u[1] = NOUT > 2 ? swap_halves_add(o[2], o[3]) : 0.f;
  return u;
}

}  // namespace pfk
