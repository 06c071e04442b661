// pa_dev.h -- device helpers shared by the gfx950 kernels: Philox4x32-10
// random words, bounded draws, ranking keys, wavefront reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

constexpr int kWave = 64;

// A pointer into global memory that the compiler cannot place (read from a
// descriptor in memory, or rebuilt from an integer) is generic, and generic
// accesses become FLAT instructions, which also count against the LDS wait
// counter: every LDS wait and workgroup barrier would then wait for the
// outstanding global traffic too.  Accesses to global memory therefore go
// through gp(p), the same pointer typed as global, which makes them global_*
// instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> gp(T *p) {
  return (gptr<T>)p;
}

// Stream tags of the counter word c3 = tag << 24 | block.
enum : uint32_t {
  kTagSelect = 0x01u,
  kTagMutDecide = 0x02u,
  kTagMutPartner = 0x03u,
  kTagInitDecide = 0x10u,
  kTagInitPartner = 0x11u,
  kTagInitShuffle = 0x12u,
};
constexpr uint32_t kInitGeneration = 0xFFFFFFFFu;  // c1 of population-init streams

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// multiplications (words 0 and 2) whose halves are swapped into place and
// xored with the round key; the key advances by the Weyl increments.
struct Words4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply per product (both halves at once)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const Words4 &b, uint32_t i) {
  return i == 0 ? b.x : i == 1 ? b.y : i == 2 ? b.z : b.w;
}

// Random stream identity: key = seed; counter = (c0, c1, c2, tag<<24 | block).
struct Stream {
  uint32_t k0, k1, c0, c1, c2, tag;
  __device__ __forceinline__ Words4 block(uint32_t b) const {
    return philox10(c0, c1, c2, (tag << 24) | b, k0, k1);
  }
  __device__ __forceinline__ uint32_t word(uint32_t i) const { return pick(block(i >> 2), i & 3u); }
};

// Lemire multiply-shift onto [0, n).
__device__ __forceinline__ uint32_t bounded(uint32_t w, uint32_t n) {
  return __umulhi(w, n);
}
// Event test against a threshold floor(p * 2^32) in [0, 2^32].
__device__ __forceinline__ bool hit(uint32_t w, uint64_t thr) { return (uint64_t)w < thr; }

// Order-preserving map of an FP32 fitness to uint32: larger key = better.
// NaN maps below everything (0); -0 and +0 get the same key.
__device__ __forceinline__ uint32_t rank_key(float f) {
  uint32_t b = __float_as_uint(f);
  if (f != f) return 0u;
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
// a beats b: larger key, or equal key and lower index.
__device__ __forceinline__ bool beats(uint32_t ka, uint32_t a, uint32_t kb, uint32_t b) {
  return ka > kb || (ka == kb && a < b);
}
// 64-bit sort key: rank key above, complemented index below (unique per index).
__device__ __forceinline__ uint64_t full_key(float f, uint32_t idx) {
  return ((uint64_t)rank_key(f) << 32) | (uint64_t)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_index(uint64_t k) { return 0xFFFFFFFFu - (uint32_t)k; }

// Wavefront reductions of 64-bit keys; every lane receives the result.  All
// 64 lanes must be active.  Within each row of 16 lanes a butterfly of DPP
// moves (quad xor 1, quad xor 2, half-row mirror, row mirror) leaves the row's
// extremum in every lane of the row; the four row results are then read from
// lanes 0, 16, 32 and 48.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL, bool MAX>
__device__ __forceinline__ void dpp_step64(uint32_t &hi, uint32_t &lo) {
  const uint32_t oh = dpp_mov<CTRL>(hi), ol = dpp_mov<CTRL>(lo);
  const bool take = MAX ? (oh > hi || (oh == hi && ol > lo)) : (oh < hi || (oh == hi && ol < lo));
  hi = take ? oh : hi;
  lo = take ? ol : lo;
}
__device__ __forceinline__ uint64_t lane_u64(uint32_t hi, uint32_t lo, int lane) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, lane) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)lo, lane);
}
template <bool MAX>
__device__ __forceinline__ uint64_t wave_reduce_u64(uint64_t v) {
  uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  dpp_step64<0xB1, MAX>(hi, lo);   // quad_perm [1,0,3,2]
  dpp_step64<0x4E, MAX>(hi, lo);   // quad_perm [2,3,0,1]
  dpp_step64<0x141, MAX>(hi, lo);  // row_half_mirror
  dpp_step64<0x140, MAX>(hi, lo);  // row_mirror
  const uint64_t r0 = lane_u64(hi, lo, 0), r1 = lane_u64(hi, lo, 16);
  const uint64_t r2 = lane_u64(hi, lo, 32), r3 = lane_u64(hi, lo, 48);
  if (MAX) {
    const uint64_t a = r0 > r1 ? r0 : r1, b = r2 > r3 ? r2 : r3;
    return a > b ? a : b;
  }
  const uint64_t a = r0 < r1 ? r0 : r1, b = r2 < r3 ? r2 : r3;
  return a < b ? a : b;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) { return wave_reduce_u64<true>(v); }
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) { return wave_reduce_u64<false>(v); }

// Byte ranges moved with aligned 32-bit loads, up to kCopyBatch loads in
// flight per thread.  A range [src, src + n) is covered by the aligned words
// w = 0 .. nwords-1 starting at src rounded down to 4 bytes; each such word
// holds at least one byte of the range, so it lies in a page the range
// touches (no fault even when the range ends at an allocation's end).
constexpr int kCopyBatch = 8;

struct ByteRange {
  const uint8_t *src;
  int n;
  __device__ __forceinline__ int words() const {
    return ((int)((uintptr_t)src & 3u) + n + 3) >> 2;
  }
  // bytes of the first aligned word before the range
  __device__ __forceinline__ int lead() const { return (int)((uintptr_t)src & 3u); }
  __device__ __forceinline__ uint32_t load(int w) const {
    return gp(reinterpret_cast<const uint32_t *>((uintptr_t)src & ~(uintptr_t)3))[w];
  }
  // byte offset in the range of byte b of word w (may fall outside [0, n))
  __device__ __forceinline__ int pos(int w, int b) const {
    return w * 4 + b - (int)((uintptr_t)src & 3u);
  }
};

// Copies [src, src + n) to dst (LDS or global, any alignment) with the whole
// workgroup.
__device__ __forceinline__ void copy_bytes(const uint8_t *src, int n, uint8_t *dst) {
  if (n <= 0) return;
  const ByteRange r{src, n};
  const int nw = r.words();
  const int step = (int)blockDim.x;
  for (int w0 = threadIdx.x; w0 < nw; w0 += kCopyBatch * step) {
    uint32_t v[kCopyBatch];
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) v[u] = r.load(min(w0 + u * step, nw - 1));
#pragma unroll
    for (int u = 0; u < kCopyBatch; ++u) {
      const int w = w0 + u * step;
      if (w < nw) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int g = r.pos(w, b);
          if (g >= 0 && g < n) dst[g] = (uint8_t)(v[u] >> (8 * b));
        }
      }
    }
  }
}

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Two-step copy of a global byte range [src, src + n) into LDS, so that the
// loads of one range can fly while the workgroup computes on the previous
// one: prefetch_issue loads this thread's aligned words (at most PF per
// thread: the range must satisfy words() <= PF * step) into registers,
// prefetch_store writes them whole to dst (LDS, 4-byte aligned): word w at
// dst + 4w, so byte i of the range lands at dst + lead() + i, and the first
// and last words carry up to 3 bytes each from outside the range (dst needs
// 4 * words() <= n + 6 bytes).  The copy is shared by `step` threads, this
// one being number t (by default the workgroup; one wave: t = lane,
// step = 64).
template <int PF>
__device__ __forceinline__ void prefetch_issue(const ByteRange &r, uint32_t (&v)[PF],
                                               int t = (int)threadIdx.x,
                                               int step = (int)blockDim.x) {
  const int nw = r.n > 0 ? r.words() : 0;
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int w = t + u * step;
    v[u] = w < nw ? r.load(w) : 0u;
  }
}
template <int PF>
__device__ __forceinline__ void prefetch_store(const ByteRange &r, const uint32_t (&v)[PF],
                                               uint8_t *dst, int t = (int)threadIdx.x,
                                               int step = (int)blockDim.x) {
  const int nw = r.n > 0 ? r.words() : 0;
#pragma unroll
  for (int u = 0; u < PF; ++u) {
    const int w = t + u * step;
    if (w < nw) reinterpret_cast<uint32_t *>(dst)[w] = v[u];
  }
}

// Copies n bytes from LDS `src` to global `dst` (any alignment) with the
// whole workgroup: 32-bit stores wherever dst is aligned, single bytes at the
// two ends.
__device__ __forceinline__ void store_bytes(uint8_t *dst, const uint8_t *src, int n) {
  if (n <= 0) return;
  const int lead = (int)((4u - ((uint32_t)(uintptr_t)dst & 3u)) & 3u);
  const int head = lead < n ? lead : n;
  const int nw = (n - head) >> 2;
  const int tail0 = head + 4 * nw;
  const int t = threadIdx.x;
  if (t < head) gp(dst)[t] = src[t];
  if (t < n - tail0) gp(dst)[tail0 + t] = src[tail0 + t];
  gptr<uint32_t> dw = gp(reinterpret_cast<uint32_t *>(dst + head));
  const uint8_t *s = src + head;
  if (((uintptr_t)s & 3u) == 0) {
    for (int w = t; w < nw; w += (int)blockDim.x) dw[w] = reinterpret_cast<const uint32_t *>(s)[w];
    return;
  }
  for (int w = t; w < nw; w += (int)blockDim.x) {
    const uint8_t *p = s + 4 * w;
    dw[w] = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
            ((uint32_t)p[3] << 24);
  }
}

}  // namespace pa
