// Memory-system probes (include/ips_probe.h): plain streaming, block moves
// between pseudo-random positions, and the block permutation's dependent
// chain (pointer atomic -> block load -> block store), each timed with HIP
// events.  Not part of sorting: they give the practical ceilings the sort's
// kernels are read against.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ips.h"
#include "../../include/ips_probe.h"

namespace {

constexpr uint32_t PT = 256;      // threads per workgroup
constexpr int U = 4;              // 16-byte accesses in flight per thread (streaming probes)
constexpr uint32_t GL = 16;       // lanes per chain group

// 32-bit integer finalizer with the multipliers of C. Wellons' "lowbias32"
// (hash-prospector); any well-mixing bijection serves.
__device__ __forceinline__ uint32_t pmix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

__global__ void __launch_bounds__(PT) k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * PT * U;
  for (uint64_t base = (uint64_t)blockIdx.x * PT * U + threadIdx.x; base < n; base += stride) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * PT;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * PT;
      if (i < n) dst[i] = v[u];
    }
  }
}

__global__ void __launch_bounds__(PT) k_probe_read(const uint4* __restrict__ src, uint32_t* sink, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * PT * U;
  uint32_t acc = 0;
  for (uint64_t base = (uint64_t)blockIdx.x * PT * U + threadIdx.x; base < n; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * PT;
      if (i < n) {
        const uint4 v = src[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;   // keeps the loads; almost never stores
}

__global__ void __launch_bounds__(PT) k_probe_write(uint4* __restrict__ dst, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * PT * U;
  for (uint64_t base = (uint64_t)blockIdx.x * PT * U + threadIdx.x; base < n; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = base + (uint64_t)u * PT;
      if (i < n) dst[i] = make_uint4((uint32_t)i, (uint32_t)(i >> 32), 1u, 2u);
    }
  }
}

// Block b of the destination receives source block (b * odd) mod nblk; the
// destination order is itself scrambled the same way with another odd
// multiplier, so both sides are bijections over the power-of-two block count.
__global__ void __launch_bounds__(PT) k_probe_blocks(const uint4* __restrict__ src, uint4* __restrict__ dst, uint64_t n,
                                                     uint32_t cb_log) {
  const uint64_t mask = (n >> cb_log) - 1, cm = (1ull << cb_log) - 1;
  const uint64_t stride = (uint64_t)gridDim.x * PT * U;
  for (uint64_t base = (uint64_t)blockIdx.x * PT * U + threadIdx.x; base < n; base += stride) {
    uint4 v[U];
    uint64_t d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t t = base + (uint64_t)u * PT;
      d[u] = 0;
      if (t < n) {
        const uint64_t blk = t >> cb_log, c = t & cm;
        const uint64_t sb = (blk * 0x9E3779B97F4A7C15ull) & mask;
        const uint64_t db = (blk * 0xD1B54A32D192ED03ull + 0x5851F42Dull) & mask;
        v[u] = src[(sb << cb_log) + c];
        d[u] = (db << cb_log) + c;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t t = base + (uint64_t)u * PT;
      if (t < n) dst[d[u]] = v[u];
    }
  }
}

// A block is GL lanes x R 16-byte units; each group runs `iters` links of
// the chain.  The loaded block's address depends on the atomic's result, so
// every link waits for one atomic and one load in turn.
template <uint32_t R>
__global__ void __launch_bounds__(PT) k_probe_chain(unsigned long long* table, uint32_t tmask, const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, uint32_t bmask, uint32_t groups,
                                                    uint32_t iters) {
  const uint32_t gtid = blockIdx.x * PT + threadIdx.x;
  const uint32_t gid = gtid / GL, gl = threadIdx.x % GL, lbase = (threadIdx.x & 63u) - gl;
  if (gid >= groups) return;   // whole groups leave together
  uint32_t h = pmix(gid * 0x9E3779B1u + 17u);
  uint32_t acc = 0;
  for (uint32_t it = 0; it < iters; ++it) {
    unsigned long long v = 0;
    if (gl == 0) v = __hip_atomic_fetch_add(&table[h & tmask], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t r = (uint32_t)__shfl((int)(uint32_t)v, (int)lbase, 64) ^ h;
    const uint64_t sb = pmix(r) & bmask, db = pmix(r ^ 0xA5A5A5A5u) & bmask;
    uint4 x[R];
#pragma unroll
    for (uint32_t q = 0; q < R; ++q) x[q] = src[sb * (GL * R) + q * GL + gl];
#pragma unroll
    for (uint32_t q = 0; q < R; ++q) dst[db * (GL * R) + q * GL + gl] = x[q];
    acc += x[0].x;
    h = pmix(h + it + 1);
  }
  if (acc == 0x9E3779B9u) dst[gl] = make_uint4(acc, 0, 0, 0);   // keeps the loads; almost never stores
}

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

uint32_t log2u(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

}  // namespace

extern "C" int ips_probe_memory(int mode, const void* src, void* dst, uint64_t bytes, uint32_t block_bytes,
                                uint64_t* table, uint32_t table_words, uint32_t groups, uint32_t reps, void* stream,
                                float* ms_per_rep) {
  if (mode < IPS_PROBE_COPY || mode > IPS_PROBE_CHAIN || !src || !dst || !ms_per_rep || reps == 0) return IPS_E_INVALID_ARG;
  if (bytes == 0 || bytes % 16 || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return IPS_E_INVALID_ARG;
  const bool blocks = mode == IPS_PROBE_BLOCKS || mode == IPS_PROBE_CHAIN;
  if (blocks) {
    if (block_bytes != 256 && block_bytes != 512 && block_bytes != 1024 && block_bytes != 2048) return IPS_E_INVALID_ARG;
    if (bytes % block_bytes || !pow2(bytes / block_bytes)) return IPS_E_INVALID_ARG;
  }
  uint32_t iters = 0;
  if (mode == IPS_PROBE_CHAIN) {
    if (!table || !pow2(table_words) || groups == 0) return IPS_E_INVALID_ARG;
    if (bytes / block_bytes > 0xFFFFFFFFull) return IPS_E_INVALID_ARG;
    const uint64_t it = bytes / ((uint64_t)groups * block_bytes);
    if (it == 0 || it > 0xFFFFFFFFull) return IPS_E_INVALID_ARG;
    iters = (uint32_t)it;
  }
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t n = bytes / 16;
  const uint64_t want = (n + PT * U - 1) / (PT * U);
  const uint32_t grid = (uint32_t)(want < 16384 ? (want ? want : 1) : 16384);
  const uint4* s4 = static_cast<const uint4*>(src);
  uint4* d4 = static_cast<uint4*>(dst);
  auto launch = [&]() -> hipError_t {
    switch (mode) {
      case IPS_PROBE_COPY:
        hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(PT), 0, st, s4, d4, n);
        break;
      case IPS_PROBE_READ:
        hipLaunchKernelGGL(k_probe_read, dim3(grid), dim3(PT), 0, st, s4, static_cast<uint32_t*>(dst), n);
        break;
      case IPS_PROBE_WRITE:
        hipLaunchKernelGGL(k_probe_write, dim3(grid), dim3(PT), 0, st, d4, n);
        break;
      case IPS_PROBE_BLOCKS:
        hipLaunchKernelGGL(k_probe_blocks, dim3(grid), dim3(PT), 0, st, s4, d4, n, log2u(block_bytes / 16));
        break;
      default: {
        const uint32_t bmask = (uint32_t)(bytes / block_bytes - 1), tmask = table_words - 1;
        const uint32_t cg = (uint32_t)(((uint64_t)groups * GL + PT - 1) / PT);
        auto* tb = reinterpret_cast<unsigned long long*>(table);
        if (block_bytes == 256)
          hipLaunchKernelGGL(k_probe_chain<1>, dim3(cg), dim3(PT), 0, st, tb, tmask, s4, d4, bmask, groups, iters);
        else if (block_bytes == 512)
          hipLaunchKernelGGL(k_probe_chain<2>, dim3(cg), dim3(PT), 0, st, tb, tmask, s4, d4, bmask, groups, iters);
        else if (block_bytes == 1024)
          hipLaunchKernelGGL(k_probe_chain<4>, dim3(cg), dim3(PT), 0, st, tb, tmask, s4, d4, bmask, groups, iters);
        else
          hipLaunchKernelGGL(k_probe_chain<8>, dim3(cg), dim3(PT), 0, st, tb, tmask, s4, d4, bmask, groups, iters);
      }
    }
    return hipGetLastError();
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (uint32_t r = 0; e == hipSuccess && r < reps; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return IPS_E_HIP;
  *ms_per_rep = ms / (float)reps;
  return IPS_OK;
}
