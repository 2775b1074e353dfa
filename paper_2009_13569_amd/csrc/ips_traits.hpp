// Element types and key orders for the gfx950 kernels.
//
// Every element is handled as DW dwords; its key is extracted from the first
// KDW dwords.  u32/u64 compare as unsigned integers; f64 keys are mapped to
// unsigned integers by the order-preserving image of IEEE 754 totalOrder
// (negative: all bits flipped; positive: sign bit set); Pair compares its
// u64 key at byte 0; the 100-byte record compares bytes 0..9 as unsigned
// bytes (Algorithm 4 of the paper with unsigned char), i.e. as a big-endian
// 80-bit integer; the Quartet compares its three u64 key words a, b, c
// lexicographically (Algorithm 3), its fourth word being payload.
//
// key_w(w) builds the key from the first KDW dwords of an element; BUF_BYTES
// is the LDS the classification's buffer blocks may take (the rest of the
// 160 KiB holds the decision tree, whose keys are largest for the Quartet).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ips {

struct K80 {
  uint64_t hi;
  uint32_t lo;
  uint32_t pad;
};

struct K192 {
  uint64_t a, b, c;
};

__device__ __forceinline__ bool kless(uint32_t a, uint32_t b) { return a < b; }
__device__ __forceinline__ bool kless(uint64_t a, uint64_t b) { return a < b; }
__device__ __forceinline__ bool kless(const K80& a, const K80& b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}
__device__ __forceinline__ bool keq(uint32_t a, uint32_t b) { return a == b; }
__device__ __forceinline__ bool keq(uint64_t a, uint64_t b) { return a == b; }
__device__ __forceinline__ bool keq(const K80& a, const K80& b) {
  return a.hi == b.hi && a.lo == b.lo;
}
__device__ __forceinline__ bool kless(const K192& x, const K192& y) {
  return x.a < y.a || (x.a == y.a && (x.b < y.b || (x.b == y.b && x.c < y.c)));
}
__device__ __forceinline__ bool keq(const K192& x, const K192& y) { return x.a == y.a && x.b == y.b && x.c == y.c; }

// c ? a : b, field by field for the composite keys (a select of whole
// structures can be lowered through private memory).
__device__ __forceinline__ uint32_t ksel(bool c, uint32_t a, uint32_t b) { return c ? a : b; }
__device__ __forceinline__ uint64_t ksel(bool c, uint64_t a, uint64_t b) { return c ? a : b; }
__device__ __forceinline__ K80 ksel(bool c, const K80& a, const K80& b) {
  K80 r;
  r.hi = c ? a.hi : b.hi;
  r.lo = c ? a.lo : b.lo;
  r.pad = 0;
  return r;
}
__device__ __forceinline__ K192 ksel(bool c, const K192& x, const K192& y) {
  K192 r;
  r.a = c ? x.a : y.a;
  r.b = c ? x.b : y.b;
  r.c = c ? x.c : y.c;
  return r;
}

constexpr uint32_t BUF_BYTES_DEFAULT = 128u * 1024u;

__device__ __forceinline__ uint64_t f64_to_ord(uint64_t b) {
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
__device__ __forceinline__ uint64_t ord_to_f64(uint64_t k) {
  return (k >> 63) ? (k & ~(1ull << 63)) : ~k;
}

struct TU32 {
  static constexpr int DW = 1, KDW = 1, CODE = 1, EPT = 12;
  static constexpr bool KEYS_ONLY = true, RADIX_OK = true;
  static constexpr uint32_t BUF_BYTES = BUF_BYTES_DEFAULT;
  using Key = uint32_t;
  __device__ static Key key(uint32_t w0, uint32_t, uint32_t) { return w0; }
  __device__ static Key key_w(const uint32_t* w) { return w[0]; }
  __device__ static Key kmax() { return 0xFFFFFFFFu; }
  __device__ static uint64_t rkey(Key k) { return k; }
  __device__ static void from_key(Key k, uint32_t* w) { w[0] = k; }
  __device__ static Key from_slot(const uint64_t* s) { return (uint32_t)s[0]; }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k; s[1] = 0; }
  // Unsigned image used to index the start-node table, and the smallest /
  // largest key whose image is x.
  __device__ static uint64_t img(Key k) { return k; }
  __device__ static Key lo_of(uint64_t x) { return (uint32_t)x; }
  __device__ static Key hi_of(uint64_t x) { return (uint32_t)x; }
  static constexpr uint64_t IMG_MAX = 0xFFFFFFFFull;
};

struct TU64 {
  static constexpr int DW = 2, KDW = 2, CODE = 2, EPT = 8;
  static constexpr bool KEYS_ONLY = true, RADIX_OK = true;
  static constexpr uint32_t BUF_BYTES = BUF_BYTES_DEFAULT;
  using Key = uint64_t;
  __device__ static Key key(uint32_t w0, uint32_t w1, uint32_t) {
    return (uint64_t)w0 | ((uint64_t)w1 << 32);
  }
  __device__ static Key key_w(const uint32_t* w) { return key(w[0], w[1], 0); }
  __device__ static Key kmax() { return ~0ull; }
  __device__ static uint64_t rkey(Key k) { return k; }
  __device__ static void from_key(Key k, uint32_t* w) { w[0] = (uint32_t)k; w[1] = (uint32_t)(k >> 32); }
  __device__ static Key from_slot(const uint64_t* s) { return s[0]; }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k; s[1] = 0; }
  __device__ static uint64_t img(Key k) { return k; }
  __device__ static Key lo_of(uint64_t x) { return x; }
  __device__ static Key hi_of(uint64_t x) { return x; }
  static constexpr uint64_t IMG_MAX = ~0ull;
};

struct TF64 {
  static constexpr int DW = 2, KDW = 2, CODE = 3, EPT = 8;
  static constexpr bool KEYS_ONLY = true, RADIX_OK = true;
  static constexpr uint32_t BUF_BYTES = BUF_BYTES_DEFAULT;
  using Key = uint64_t;
  __device__ static Key key(uint32_t w0, uint32_t w1, uint32_t) {
    return f64_to_ord((uint64_t)w0 | ((uint64_t)w1 << 32));
  }
  __device__ static Key key_w(const uint32_t* w) { return key(w[0], w[1], 0); }
  __device__ static Key kmax() { return ~0ull; }
  __device__ static uint64_t rkey(Key k) { return k; }
  __device__ static void from_key(Key k, uint32_t* w) {
    uint64_t b = ord_to_f64(k);
    w[0] = (uint32_t)b; w[1] = (uint32_t)(b >> 32);
  }
  __device__ static Key from_slot(const uint64_t* s) { return s[0]; }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k; s[1] = 0; }
  __device__ static uint64_t img(Key k) { return k; }
  __device__ static Key lo_of(uint64_t x) { return x; }
  __device__ static Key hi_of(uint64_t x) { return x; }
  static constexpr uint64_t IMG_MAX = ~0ull;
};

struct TPair {
  static constexpr int DW = 4, KDW = 2, CODE = 4, EPT = 4;
  static constexpr bool KEYS_ONLY = false, RADIX_OK = true;
  static constexpr uint32_t BUF_BYTES = BUF_BYTES_DEFAULT;
  using Key = uint64_t;
  __device__ static Key key(uint32_t w0, uint32_t w1, uint32_t) {
    return (uint64_t)w0 | ((uint64_t)w1 << 32);
  }
  __device__ static Key key_w(const uint32_t* w) { return key(w[0], w[1], 0); }
  __device__ static Key kmax() { return ~0ull; }
  __device__ static uint64_t rkey(Key k) { return k; }
  __device__ static Key from_slot(const uint64_t* s) { return s[0]; }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k; s[1] = 0; }
  __device__ static uint64_t img(Key k) { return k; }
  __device__ static Key lo_of(uint64_t x) { return x; }
  __device__ static Key hi_of(uint64_t x) { return x; }
  static constexpr uint64_t IMG_MAX = ~0ull;
};

struct TRec100 {
  static constexpr int DW = 25, KDW = 3, CODE = 5, EPT = 1;
  static constexpr bool KEYS_ONLY = false, RADIX_OK = false;
  static constexpr uint32_t BUF_BYTES = BUF_BYTES_DEFAULT;
  using Key = K80;
  __device__ static Key key(uint32_t w0, uint32_t w1, uint32_t w2) {
    K80 k;
    k.hi = ((uint64_t)__builtin_bswap32(w0) << 32) | (uint64_t)__builtin_bswap32(w1);
    k.lo = ((w2 & 0xFFu) << 8) | ((w2 >> 8) & 0xFFu);
    k.pad = 0;
    return k;
  }
  __device__ static Key key_w(const uint32_t* w) { return key(w[0], w[1], w[2]); }
  __device__ static Key kmax() { K80 k; k.hi = ~0ull; k.lo = 0xFFFFu; k.pad = 0; return k; }
  __device__ static uint64_t rkey(Key) { return 0; }
  __device__ static Key from_slot(const uint64_t* s) {
    K80 k; k.hi = s[0]; k.lo = (uint32_t)s[1]; k.pad = 0; return k;
  }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k.hi; s[1] = k.lo; }
  __device__ static uint64_t img(Key k) { return k.hi; }
  __device__ static Key lo_of(uint64_t x) { K80 k; k.hi = x; k.lo = 0; k.pad = 0; return k; }
  __device__ static Key hi_of(uint64_t x) { K80 k; k.hi = x; k.lo = 0xFFFFu; k.pad = 0; return k; }
  static constexpr uint64_t IMG_MAX = ~0ull;
};

// Quartet: 32 bytes, key words a, b, c at bytes 0, 8, 16, payload at 24.
struct TQuartet {
  static constexpr int DW = 8, KDW = 6, CODE = 6, EPT = 2;
  static constexpr bool KEYS_ONLY = false, RADIX_OK = false;
  static constexpr uint32_t BUF_BYTES = 120u * 1024u;
  using Key = K192;
  __device__ static Key key_w(const uint32_t* w) {
    K192 k;
    k.a = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    k.b = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    k.c = (uint64_t)w[4] | ((uint64_t)w[5] << 32);
    return k;
  }
  __device__ static Key kmax() { K192 k; k.a = ~0ull; k.b = ~0ull; k.c = ~0ull; return k; }
  __device__ static uint64_t rkey(Key) { return 0; }
  __device__ static Key from_slot(const uint64_t* s) { K192 k; k.a = s[0]; k.b = s[1]; k.c = s[2]; return k; }
  __device__ static void to_slot(Key k, uint64_t* s) { s[0] = k.a; s[1] = k.b; s[2] = k.c; }
  __device__ static uint64_t img(Key k) { return k.a; }
  __device__ static Key lo_of(uint64_t x) { K192 k; k.a = x; k.b = 0; k.c = 0; return k; }
  __device__ static Key hi_of(uint64_t x) { K192 k; k.a = x; k.b = ~0ull; k.c = ~0ull; return k; }
  static constexpr uint64_t IMG_MAX = ~0ull;
};

}  // namespace ips
