// Lane moves and reductions of a wave64 tile (lane = jl * 8 + il), shared by
// the tile kernel and the backward parameter pass.
#pragma once
#include <hip/hip_runtime.h>

namespace anb {

// sum over the 8 lanes of each lane group (lane & ~7): quad_perm xor 1, xor 2, row_half_mirror
// (every source lane exists, so bound_ctrl changes nothing but lets the
// compiler fold each lane move into its add)
__device__ inline float red8(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
  return v;
}
__device__ inline double dpp_d(double v, int ctrl) {
  const long long b = __double_as_longlong(v);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  if (ctrl == 0xB1) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else if (ctrl == 0x4E) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double red8(double v) {
  v += dpp_d(v, 0xB1);
  v += dpp_d(v, 0x4E);
  v += dpp_d(v, 0x141);
  return v;
}
// sum over lanes with equal (lane & 7): xor 8, 16, 32
template <typename R>
__device__ inline R red_jl(R v) {
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}
// Reduce-scatter of the i-forces over jl: in[c] is lane (jl, il)'s
// contribution to atom il of i-cluster c; the result in lane (jl, il) is
// the sum over jl of in[jl], i.e. the total for slot c * 8 + il with c = jl.
// Three halving steps: lanes 32 apart (jl bit 2) with v_permlane32_swap,
// 16 apart (jl bit 1) with v_permlane16_swap, 8 apart (jl bit 0) with a
// row rotation by 8.
__device__ inline void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ inline void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}
__device__ inline void swap32(double& a, double& b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ inline void swap16(double& a, double& b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)y, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(y >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ inline float ror8(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, true));
}
__device__ inline double ror8(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x128, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x128, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename R>
__device__ inline R scatter_jl(R (&in)[8], bool odd8) {
  R p[4], q[2];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R a = in[c], b = in[c + 4];
    swap32(a, b);
    p[c] = a + b;  // lanes 0-31: cluster c; lanes 32-63: cluster c + 4
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    R a = p[c], b = p[c + 2];
    swap16(a, b);
    q[c] = a + b;  // even rows: + 0; odd rows: + 2
  }
  const R keep = odd8 ? q[1] : q[0], send = odd8 ? q[0] : q[1];
  return keep + ror8(send);
}

}  // namespace anb
