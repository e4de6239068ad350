// Issue-rate microbenchmark for gfx950: eight independent dependency chains
// per lane of one instruction type (FP32 FMA, MUL, and the transcendentals
// sin/rsq/exp2/rcp that the Green's-term kernels use), timed with HIP
// events over five launches of 8192 blocks x 256 threads.  Prints lane
// instructions per second and the ratio to 256 CU x 64 lanes x 2.4 GHz.
// Built by paper_2102_02738_amd/build.py as diag/valu_rate.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#define CH 8
#define IT 2048
template <int OP>
__global__ __launch_bounds__(256) void k(float* out, float seed) {
  float v[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) v[c] = seed + 0.001f * (threadIdx.x + c);
  for (int i = 0; i < IT; ++i) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (OP == 0) v[c] = fmaf(v[c], 0.999f, 0.0001f);
      if (OP == 1) v[c] = __builtin_amdgcn_sinf(v[c]);
      if (OP == 2) v[c] = __builtin_amdgcn_rsqf(v[c]);
      if (OP == 3) v[c] = __builtin_amdgcn_exp2f(v[c]);
      if (OP == 4) v[c] = __builtin_amdgcn_rcpf(v[c]);
      if (OP == 5) { v[c] = __builtin_amdgcn_sinf(v[c]); v[c] = fmaf(v[c], 0.999f, 0.0001f); v[c] = fmaf(v[c], 0.999f, 0.0001f); v[c] = fmaf(v[c], 0.999f, 0.0001f);}
      if (OP == 6) v[c] = v[c] * 0.999f;
    }
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < CH; ++c) s += v[c];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
static void chk(hipError_t e) {
  if (e != hipSuccess) { fprintf(stderr, "HIP error: %s\n", hipGetErrorString(e)); exit(1); }
}
template <int OP> double run(float* d, int blocks) {
  hipEvent_t a, b;
  chk(hipEventCreate(&a)); chk(hipEventCreate(&b));
  hipLaunchKernelGGL(k<OP>, dim3(blocks), dim3(256), 0, 0, d, 0.3f);
  chk(hipGetLastError());
  chk(hipEventRecord(a));
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k<OP>, dim3(blocks), dim3(256), 0, 0, d, 0.3f);
  chk(hipGetLastError());
  chk(hipEventRecord(b)); chk(hipEventSynchronize(b));
  float ms; chk(hipEventElapsedTime(&ms, a, b));
  chk(hipEventDestroy(a)); chk(hipEventDestroy(b));
  double ops = 5.0 * blocks * 256.0 * CH * IT * (OP == 5 ? 4 : 1);
  return ops / (ms * 1e-3);
}
int main() {
  int blocks = 256 * 32;
  float* d; if (hipMalloc(&d, blocks * 256 * 4)) return 2;
  const char* names[] = {"fma", "sin", "rsq", "exp2", "rcp", "sin+3fma", "mul"};
  double r[7];
  r[0] = run<0>(d, blocks); r[1] = run<1>(d, blocks); r[2] = run<2>(d, blocks); r[3] = run<3>(d, blocks);
  r[4] = run<4>(d, blocks); r[5] = run<5>(d, blocks); r[6] = run<6>(d, blocks);
  for (int i = 0; i < 7; ++i) printf("%-10s %.3e lane-instr/s  (%.3f of 3.93e13)\n", names[i], r[i], r[i] / 3.93216e13);
  hipDeviceProp_t p; chk(hipGetDeviceProperties(&p, 0));
  printf("CUs %d clock %d kHz\n", p.multiProcessorCount, p.clockRate);
  return hipDeviceSynchronize() != hipSuccess;
}
