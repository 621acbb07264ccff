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

// Piece-local contact index of this lane's survivor in tile j of entry E, or
// -1 past the entry's last survivor.
CM_DEV int tile_contact(const uint64_t* __restrict__ bits, const Entry& E, int j) {
  const int r0 = j * kWave, r = r0 + lane();
  const int nw = (max(E.count, 0) + kWave - 1) / kWave;
  const uint64_t* wp = bits + E.word_off;
  int pre = 0, c = -1;
  for (int w = 0; w < nw && pre < r0 + kWave; ++w) {
    const uint64_t word = wp[w];
    const int pc = __popcll(word);
    if (pre + pc > r0 && r >= pre && r < pre + pc) c = w * kWave + kth_bit(word, r - pre);
    pre += pc;
  }
  return c;
}

// Entry of tile t: the largest e with tile_off[e] <= t.
CM_DEV int64_t find_entry(const int64_t* __restrict__ tile_off, int64_t n_ent, int64_t t) {
  int64_t lo = 0, hi = n_ent;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (tile_off[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

CM_DEV V3<float> vert(const ObjDesc& o, int i) { return {o.vx[i], o.vy[i], o.vz[i]}; }

}  // namespace cm
