// probe.hip -- a kernel of known vector-ALU work, outside the map path.
//
// Hardware instruction counters (rocprofv3 SQ_INSTS_VALU_*) and the vector
// ALU's issue rate are read against it: every lane runs `iters` iterations
// of 16 independent fused multiply-adds, so a launch of `blocks` workgroups
// of 256 threads issues exactly blocks * 4 * iters * 16 FMA instructions per
// wavefront count (plus 15 adds per wavefront for the final sum), and
// 2 * 64 times that many FLOP.  The 16 chains are independent, so the
// instruction stream is limited by issue rather than by latency.  The
// multiplier and addend are uniform; by default they are copied into vector
// registers first, since on gfx950 an FP32 FMA that reads a scalar register
// issues at about half the rate of one with vector operands only (the third
// kind keeps the multiplier in a scalar register to show this).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csmap {

namespace {

constexpr int kProbeChains = 16;

__device__ __forceinline__ float vreg(float x) {
  float y;
  asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
  return y;
}

__device__ __forceinline__ double vreg(double x) {
  double y;
  asm volatile("v_mov_b64 %0, %1" : "=v"(y) : "s"(x));
  return y;
}

template <typename T, bool kScalarMul>
__global__ void __launch_bounds__(256) k_valu_probe(int64_t iters, T m_arg, T c_arg, T* out) {
  const T c = vreg(c_arg);
  const T m = kScalarMul ? m_arg : vreg(m_arg);
  T a[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) a[k] = (T)(threadIdx.x + k);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = fma(a[k], m, c);
  }
  T s = a[0];
#pragma unroll
  for (int k = 1; k < kProbeChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// kind 0: FP32 (v_fma_f32), vector operands; 1: FP64 (v_fma_f64), vector
// operands; 2: FP32 with the multiplier in a scalar register.
hipError_t launch_valu_probe(int kind, int64_t blocks, int64_t iters, void* out, hipStream_t st) {
  const dim3 grid((unsigned)blocks), block(256);
  if (kind == 0)
    k_valu_probe<float, false><<<grid, block, 0, st>>>(iters, 0.999f, 0.001f, (float*)out);
  else if (kind == 1)
    k_valu_probe<double, false><<<grid, block, 0, st>>>(iters, 0.999, 0.001, (double*)out);
  else
    k_valu_probe<float, true><<<grid, block, 0, st>>>(iters, 0.999f, 0.001f, (float*)out);
  return hipGetLastError();
}

int64_t valu_probe_chains() { return kProbeChains; }

}  // namespace csmap
