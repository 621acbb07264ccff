// Wave-level helpers and work-queue decoding shared by the gfx950 kernels.
#pragma once
#include "devmath.h"

namespace cm {

CM_DEV int lane() { return int(threadIdx.x) & (kWave - 1); }
CM_DEV float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
CM_DEV df wsum(df v) { return {wsum(v.v), wsum(v.t)}; }
CM_DEV float wmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}
CM_DEV int wmax_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
  return v;
}
CM_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Index of the k-th set bit (k counted from 0) of a 64-bit word.
CM_DEV int kth_bit(uint64_t w, int k) {
  int pos = 0;
#pragma unroll
  for (int s = 32; s >= 1; s >>= 1) {
    const uint64_t low = w & ((uint64_t(1) << s) - 1);
    const int c = __popcll(low);
    if (k >= c) { k -= c; w >>= s; pos += s; } else { w = low; }
  }
  return pos;
}

// Largest index i in [lo, hi) with off[i] <= v (off non-decreasing, off[lo] <= v).
CM_DEV int64_t last_le(const int64_t* __restrict__ off, int64_t lo, int64_t hi, int64_t v) {
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// Entry-local index of the k-th survivor (k counted from 0) of entry E: the
// word holding it from the per-word survivor prefix, then the bit in the word.
CM_DEV int entry_survivor(const uint64_t* __restrict__ bits, const int32_t* __restrict__ wpre, const Entry& E, int k) {
  const int nw = (max(E.count, 0) + kWave - 1) / kWave;
  int lo = 0, hi = nw;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (wpre[E.word_off + mid] <= k) lo = mid; else hi = mid;
  }
  return lo * kWave + kth_bit(bits[E.word_off + lo], k - wpre[E.word_off + lo]);
}

CM_DEV V3<float> vert(const ObjDesc& o, int i) { return {o.vx[i], o.vy[i], o.vz[i]}; }

}  // namespace cm
