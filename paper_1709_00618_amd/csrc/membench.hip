// Memory-system ceilings for random accesses on one GPU: random 8-B loads
// (with each load cache policy), scattered stores of 4..128 B, and random
// atomicMax on 32- and 64-bit words.  The tracker's fit and selection make
// exactly these accesses (one track per lane, one pad row per step), so
// these rates, not HBM bandwidth for streaming, are their ceilings.
// Every address is reduced modulo its table's size: all accesses stay in
// bounds.  Output: one line per measurement.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

namespace {

__device__ __forceinline__ unsigned long long mix(unsigned long long x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 29;
  return x;
}

// kAux < 0: a plain global load; otherwise a buffer load with these
// cache-policy bits (1 sc0, 2 nt, 16 sc1).
template <int kAux>
__global__ void k_gather(const unsigned long long *a, unsigned long long n, unsigned long long *out, int iters) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  // a buffer resource over the first 2 GiB - 1 of the table
  __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)a, 0, 0x7FFFFFFF, 0x00020000);
  unsigned long long x = tid * 0x9E3779B97F4A7C15ull + 1, acc = 0;
  for (int it = 0; it < iters; ++it) {
    x = mix(x);
    const unsigned long long i = x % n;  // n * 8 B <= 2 GiB
    if (kAux < 0) {
      acc += a[i];
    } else {
      const auto r = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(i * 8u), 0, kAux);
      acc += ((unsigned long long)r[1] << 32) | r[0];
    }
  }
  out[tid] = acc;
}

// kWords 32-bit words per lane into a random 128-B line, aligned to their size
template <int kWords>
__global__ void k_scatter(unsigned int *a, unsigned long long nlines, int iters) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  unsigned long long x = tid * 0x9E3779B97F4A7C15ull + 7;
  for (int it = 0; it < iters; ++it) {
    x = mix(x);
    const unsigned long long line = x % nlines;
    const unsigned int off = (unsigned int)(x >> 40) % (32 / kWords) * kWords;
    unsigned int *p = a + line * 32 + off;
#pragma unroll
    for (int w = 0; w < kWords; ++w) p[w] = (unsigned int)it;
  }
}

template <typename T>
__global__ void k_amax(T *a, unsigned long long n, int iters) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  unsigned long long x = tid * 0x9E3779B97F4A7C15ull + 3;
  for (int it = 0; it < iters; ++it) {
    x = mix(x);
    atomicMax(&a[x % n], (T)(x >> 3));
  }
}

// The XCD (XCC) the wave runs on, from the hardware register.
__device__ __forceinline__ unsigned xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u; }

// Each XCD updates its own region of n_per words with workgroup-scope
// atomics (no other XCD touches the region, so the result is the same as
// with device-scope atomics): would a claim scheme that keeps each sector's
// claims on one XCD run its atomics faster?
template <typename T>
__global__ void k_amax_xcd(T *a, unsigned long long n_per, int iters) {
  const unsigned long long tid = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
  T *r = a + xcc_id() * n_per;
  unsigned long long x = tid * 0x9E3779B97F4A7C15ull + 3;
  for (int it = 0; it < iters; ++it) {
    x = mix(x);
    __hip_atomic_fetch_max(&r[x % n_per], (T)(x >> 3), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// XCD of every block (for the block-to-XCD mapping)
__global__ void k_xcc(unsigned *o) {
  if (threadIdx.x == 0) o[blockIdx.x] = xcc_id();
}

bool ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "membench: %s: %s\n", what, hipGetErrorString(e));
  return false;
}

}  // namespace

int main() {
  const int blocks = 256 * 32, threads = 256;
  const unsigned long long table = 1ull << 31;  // 2 GiB
  void *buf = nullptr, *out = nullptr;
  if (!ok(hipMalloc(&buf, table), "hipMalloc") ||
      !ok(hipMalloc(&out, (size_t)blocks * threads * 8), "hipMalloc"))
    return 1;
  if (!ok(hipMemset(buf, 0, table), "hipMemset")) return 1;
  hipEvent_t e0, e1;
  if (!ok(hipEventCreate(&e0), "event") || !ok(hipEventCreate(&e1), "event")) return 1;
  // one warm launch, then 5 timed; prints the rate of the timed launches
  auto time_it = [&](const char *what, double per_launch, auto launch) -> bool {
    launch();
    if (!ok(hipDeviceSynchronize(), what)) return false;
    (void)hipEventRecord(e0);
    for (int r = 0; r < 5; ++r) launch();
    (void)hipEventRecord(e1);
    if (!ok(hipEventSynchronize(e1), what)) return false;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    std::printf("%-44s %9.3f ms per launch  %7.2f G/s\n", what, ms / 5, per_launch / (ms / 5 * 1e-3) / 1e9);
    std::fflush(stdout);
    return true;
  };
  const unsigned long long n64 = table / 8;
  auto *a64 = static_cast<unsigned long long *>(buf);
  auto *o64 = static_cast<unsigned long long *>(out);
  const double g = (double)blocks * threads * 64;
  bool good = true;
  good = good && time_it("random 8-B load, plain (2 GiB)", g, [&] { k_gather<-1><<<blocks, threads>>>(a64, n64, o64, 64); });
  good = good && time_it("random 8-B load, buffer, sc0", g, [&] { k_gather<1><<<blocks, threads>>>(a64, n64, o64, 64); });
  good = good && time_it("random 8-B load, buffer, nt", g, [&] { k_gather<2><<<blocks, threads>>>(a64, n64, o64, 64); });
  good = good && time_it("random 8-B load, buffer, sc1", g, [&] { k_gather<16><<<blocks, threads>>>(a64, n64, o64, 64); });
  good = good && time_it("random 8-B load, buffer, sc0 sc1", g, [&] { k_gather<17><<<blocks, threads>>>(a64, n64, o64, 64); });
  // the same over tables that fit the 256 MB last-level cache (MALL) and L2
  good = good && time_it("random 8-B load, plain (128 MiB)", g, [&] { k_gather<-1><<<blocks, threads>>>(a64, n64 / 16, o64, 64); });
  good = good && time_it("random 8-B load, plain (32 MiB)", g, [&] { k_gather<-1><<<blocks, threads>>>(a64, n64 / 64, o64, 64); });
  good = good && time_it("random 8-B load, plain (2 MiB)", g, [&] { k_gather<-1><<<blocks, threads>>>(a64, n64 / 1024, o64, 64); });
  auto *a32 = static_cast<unsigned int *>(buf);
  const unsigned long long nl = table / 128;
  const double sc = (double)blocks * threads * 16;
  good = good && time_it("scattered store, 4 B (2 GiB)", sc, [&] { k_scatter<1><<<blocks, threads>>>(a32, nl, 16); });
  good = good && time_it("scattered store, 16 B", sc, [&] { k_scatter<4><<<blocks, threads>>>(a32, nl, 16); });
  good = good && time_it("scattered store, 32 B", sc, [&] { k_scatter<8><<<blocks, threads>>>(a32, nl, 16); });
  good = good && time_it("scattered store, 64 B", sc, [&] { k_scatter<16><<<blocks, threads>>>(a32, nl, 16); });
  good = good && time_it("scattered store, 128 B", sc, [&] { k_scatter<32><<<blocks, threads>>>(a32, nl, 16); });
  const unsigned long long small = 1ull << 28;  // 256 MiB, the size of the owner words of a time frame
  const double am = (double)blocks * threads * 8;
  good = good && time_it("random atomicMax, 32-bit (256 MiB)", am,
                         [&] { k_amax<unsigned int><<<blocks, threads>>>(a32, small / 4, 8); });
  good = good && time_it("random atomicMax, 64-bit (256 MiB)", am,
                         [&] { k_amax<unsigned long long><<<blocks, threads>>>(a64, small / 8, 8); });
  good = good && time_it("random atomicMax, 32-bit (128 MiB)", am,
                         [&] { k_amax<unsigned int><<<blocks, threads>>>(a32, small / 8, 8); });
  good = good && time_it("random atomicMax, 64-bit (128 MiB)", am,
                         [&] { k_amax<unsigned long long><<<blocks, threads>>>(a64, small / 16, 8); });
  good = good && time_it("random atomicMax, 32-bit (32 MiB)", am,
                         [&] { k_amax<unsigned int><<<blocks, threads>>>(a32, small / 32, 8); });
  good = good && time_it("random atomicMax, 32-bit (2 MiB)", am,
                         [&] { k_amax<unsigned int><<<blocks, threads>>>(a32, small / 512, 8); });
  // per-XCD regions (8 x the size) with L2 atomics
  good = good && time_it("atomicMax 64-bit, wg scope, 2 MiB per XCD", am,
                         [&] { k_amax_xcd<unsigned long long><<<blocks, threads>>>(a64, (2ull << 20) / 8, 8); });
  good = good && time_it("atomicMax 64-bit, wg scope, 8 MiB per XCD", am,
                         [&] { k_amax_xcd<unsigned long long><<<blocks, threads>>>(a64, (8ull << 20) / 8, 8); });
  good = good && time_it("atomicMax 64-bit, wg scope, 32 MiB per XCD", am,
                         [&] { k_amax_xcd<unsigned long long><<<blocks, threads>>>(a64, (32ull << 20) / 8, 8); });
  good = good && time_it("atomicMax 32-bit, wg scope, 32 MiB per XCD", am,
                         [&] { k_amax_xcd<unsigned int><<<blocks, threads>>>(a32, (32ull << 20) / 4, 8); });
  if (good) {
    auto *o32 = static_cast<unsigned *>(out);
    k_xcc<<<blocks, 64>>>(o32);
    std::vector<unsigned> ids(blocks);
    good = ok(hipMemcpy(ids.data(), o32, blocks * sizeof(unsigned), hipMemcpyDeviceToHost), "xcc ids");
    int cnt[8] = {0}, rr = 0;
    for (int b = 0; b < blocks; ++b) {
      ++cnt[ids[b] & 7];
      rr += (int)(ids[b] == (unsigned)(b & 7));
    }
    std::printf("blocks per XCC:");
    for (int q = 0; q < 8; ++q) std::printf(" %d", cnt[q]);
    std::printf("; XCC == blockIdx %% 8 for %d of %d\n", rr, blocks);
  }
  (void)hipFree(buf);
  (void)hipFree(out);
  return good ? 0 : 1;
}
