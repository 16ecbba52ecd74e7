// LDS read-bandwidth probe for the roofline of the LDS-heavy kernels.  Every block
// fills 32 KiB of LDS once; then, per iteration, each of its 256 threads reads the
// whole buffer back in 16-byte (8 loads) or 8-byte (16 loads) vector loads, lane l
// at byte 16 l (or 8 l) plus an immediate offset: consecutive lanes read consecutive
// addresses, so there are no bank conflicts.  The loads and the wait for them are one
// volatile assembly statement, so that the compiler can neither hoist, merge nor
// narrow them; one add per load keeps the vector ALU far below the LDS rate.  Measurement only: the stereo library does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kBytes = 32768;

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// One iteration of one thread: the eight 16-byte or sixteen 8-byte loads and the wait
// for them, in one statement, into distinct registers that are read only after it.
__device__ __forceinline__ float read_all16(uint32_t a) {
  f4 v0, v1, v2, v3, v4, v5, v6, v7;
  asm volatile(
      "ds_read_b128 %0, %8 offset:0\n\t"
      "ds_read_b128 %1, %8 offset:4096\n\t"
      "ds_read_b128 %2, %8 offset:8192\n\t"
      "ds_read_b128 %3, %8 offset:12288\n\t"
      "ds_read_b128 %4, %8 offset:16384\n\t"
      "ds_read_b128 %5, %8 offset:20480\n\t"
      "ds_read_b128 %6, %8 offset:24576\n\t"
      "ds_read_b128 %7, %8 offset:28672\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5), "=&v"(v6), "=&v"(v7)
      : "v"(a)
      : "memory");
  return ((v0[0] + v1[0]) + (v2[0] + v3[0])) + ((v4[0] + v5[0]) + (v6[0] + v7[0]));
}

__device__ __forceinline__ float read_all8(uint32_t a) {
  f2 v0, v1, v2, v3, v4, v5, v6, v7, w0, w1, w2, w3, w4, w5, w6, w7;
  asm volatile(
      "ds_read_b64 %0, %16 offset:0\n\t"
      "ds_read_b64 %1, %16 offset:2048\n\t"
      "ds_read_b64 %2, %16 offset:4096\n\t"
      "ds_read_b64 %3, %16 offset:6144\n\t"
      "ds_read_b64 %4, %16 offset:8192\n\t"
      "ds_read_b64 %5, %16 offset:10240\n\t"
      "ds_read_b64 %6, %16 offset:12288\n\t"
      "ds_read_b64 %7, %16 offset:14336\n\t"
      "ds_read_b64 %8, %16 offset:16384\n\t"
      "ds_read_b64 %9, %16 offset:18432\n\t"
      "ds_read_b64 %10, %16 offset:20480\n\t"
      "ds_read_b64 %11, %16 offset:22528\n\t"
      "ds_read_b64 %12, %16 offset:24576\n\t"
      "ds_read_b64 %13, %16 offset:26624\n\t"
      "ds_read_b64 %14, %16 offset:28672\n\t"
      "ds_read_b64 %15, %16 offset:30720\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5), "=&v"(v6), "=&v"(v7),
        "=&v"(w0), "=&v"(w1), "=&v"(w2), "=&v"(w3), "=&v"(w4), "=&v"(w5), "=&v"(w6), "=&v"(w7)
      : "v"(a)
      : "memory");
  return ((v0[0] + v1[0]) + (v2[0] + v3[0])) + ((v4[0] + v5[0]) + (v6[0] + v7[0])) +
         (((w0[0] + w1[0]) + (w2[0] + w3[0])) + ((w4[0] + w5[0]) + (w6[0] + w7[0])));
}

template <int W>
__global__ __launch_bounds__(kThreads) void lds_read_kernel(int iters, float* out) {
  __shared__ __align__(16) float buf[kBytes / 4];
  for (int i = threadIdx.x; i < kBytes / 4; i += kThreads) buf[i] = static_cast<float>(i & 255);
  __syncthreads();
  typedef const __attribute__((address_space(3))) char* lds_ptr;
  // lane address: byte W * tid; the largest load ends at (kBytes / W / 256 - 1) *
  // 256 W + 255 W + W = kBytes
  const uint32_t a = static_cast<uint32_t>(reinterpret_cast<uintptr_t>((lds_ptr)buf)) + W * threadIdx.x;
  float acc = 0.f;
  for (int it = 0; it < iters; ++it) acc += W == 16 ? read_all16(a) : read_all8(a);
  if (acc == -1.f) out[blockIdx.x * kThreads + threadIdx.x] = acc;  // never true; keeps the sum live
}

}  // namespace

// Launches `blocks` blocks of 256 threads; each thread reads 32 KiB per iteration from
// LDS, `iters` iterations, in loads of `width` bytes (8 or 16).  out: device buffer of
// blocks * 256 floats (written only if the sums take an impossible value).  Returns 0,
// or -1 for a bad argument, -2 for a launch error.
extern "C" int rsv_probe_lds_read(int width, int blocks, int iters, float* out, void* stream) {
  if (!out || blocks < 1 || iters < 1 || (width != 8 && width != 16)) return -1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (width == 8)
    lds_read_kernel<8><<<dim3(blocks), dim3(kThreads), 0, st>>>(iters, out);
  else
    lds_read_kernel<16><<<dim3(blocks), dim3(kThreads), 0, st>>>(iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
