// isrsgn_peaks: issue-rate and accuracy microbenchmarks of the gfx950 VALU operations the pair
// integral is built from (FP32 FMA, FP64 FMA, v_sin_f32 / v_exp_f32, FP64 phase reduction).
// Prints lanes per clock per CU for each operation and the accuracy of the hardware sine,
// cosine (arguments in revolutions) and exp2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

namespace {

constexpr int kChains = 8;
constexpr int kIters = 4096;

template <int OP>
__global__ void __launch_bounds__(256) k_rate(float* out, float seed) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  float x[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = seed * (gid + c + 1) * 1e-7f;
    d[c] = x[c];
  }
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if (OP == 0) x[c] = __builtin_amdgcn_sinf(x[c]);
      if (OP == 1) x[c] = __builtin_amdgcn_exp2f(x[c]);
      if (OP == 2) x[c] = __builtin_fmaf(x[c], 0.999f, 1e-3f);
      if (OP == 3) d[c] = __builtin_fma(d[c], 0.999, 1e-3);
      if (OP == 4) { const double t = d[c] * 1.0000001; d[c] = t - __builtin_rint(t); }  // phase reduction
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c] + (float)d[c];
  out[gid] = s;
}

template <int OP>
double rate(float* dout, int grid, int block, int cus, double clk_hz) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  hipLaunchKernelGGL(k_rate<OP>, dim3(grid), dim3(block), 0, 0, dout, 1.0f);
  (void)hipEventRecord(a);
  for (int r = 0; r < 5; ++r) hipLaunchKernelGGL(k_rate<OP>, dim3(grid), dim3(block), 0, 0, dout, 1.0f);
  (void)hipEventRecord(b);
  (void)hipEventSynchronize(b);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  const double ops = 5.0 * grid * (double)block * kIters * kChains * (OP == 4 ? 2.0 : 1.0);
  return ops / (ms * 1e-3) / (cus * clk_hz);
}

__global__ void k_accuracy(const float* x, float* s, float* c, float* e, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  s[i] = __builtin_amdgcn_sinf(x[i]);
  c[i] = __builtin_amdgcn_cosf(x[i]);
  e[i] = __builtin_amdgcn_exp2f(x[i] * 40.0f);
}

}  // namespace

int main() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    std::fprintf(stderr, "no HIP device\n");
    return 1;
  }
  const int cus = p.multiProcessorCount, block = 256, grid = cus * 16;
  const double clk = p.clockRate * 1e3;
  std::printf("device %s, %d CUs, %.0f MHz\n", p.gcnArchName, cus, clk / 1e6);
  float* dout = nullptr;
  if (hipMalloc(&dout, sizeof(float) * grid * block) != hipSuccess) return 1;
  std::printf("lanes per clock per CU: v_sin_f32 %.1f  v_exp_f32 %.1f  v_fma_f32 %.1f  v_fma_f64 %.1f  "
              "f64 mul+rndne+sub %.1f\n",
              rate<0>(dout, grid, block, cus, clk), rate<1>(dout, grid, block, cus, clk),
              rate<2>(dout, grid, block, cus, clk), rate<3>(dout, grid, block, cus, clk),
              rate<4>(dout, grid, block, cus, clk));
  (void)hipFree(dout);

  const int n = 1 << 16;
  std::vector<float> x(n), s(n), c(n), e(n);
  float *dx = nullptr, *ds = nullptr, *dc = nullptr, *de = nullptr;
  if (hipMalloc(&dx, n * 4) != hipSuccess || hipMalloc(&ds, n * 4) != hipSuccess || hipMalloc(&dc, n * 4) != hipSuccess ||
      hipMalloc(&de, n * 4) != hipSuccess)
    return 1;
  auto run = [&]() {
    (void)hipMemcpy(dx, x.data(), n * 4, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k_accuracy, dim3(n / 256), dim3(256), 0, 0, dx, ds, dc, de, n);
    (void)hipMemcpy(s.data(), ds, n * 4, hipMemcpyDeviceToHost);
    (void)hipMemcpy(c.data(), dc, n * 4, hipMemcpyDeviceToHost);
    (void)hipMemcpy(e.data(), de, n * 4, hipMemcpyDeviceToHost);
  };
  for (int i = 0; i < n; ++i) x[i] = -0.5f + (float)i / n;
  run();
  double ws = 0, wc = 0, we = 0;
  for (int i = 0; i < n; ++i) {
    ws = std::fmax(ws, std::fabs(s[i] - std::sin(2 * M_PI * (double)x[i])));
    wc = std::fmax(wc, std::fabs(c[i] - std::cos(2 * M_PI * (double)x[i])));
    const double r = std::exp2((double)x[i] * 40.0);
    we = std::fmax(we, std::fabs(e[i] - r) / r);
  }
  std::printf("revolutions in [-1/2, 1/2): max |sin err| %.2e, max |cos err| %.2e; exp2 on [-20, 20): max rel %.2e\n",
              ws, wc, we);
  // the same over one full turn [0, 1): the hardware reduces its argument itself
  for (int i = 0; i < n; ++i) x[i] = (float)i / n;
  run();
  ws = wc = 0;
  for (int i = 0; i < n; ++i) {
    ws = std::fmax(ws, std::fabs(s[i] - std::sin(2 * M_PI * (double)x[i])));
    wc = std::fmax(wc, std::fabs(c[i] - std::cos(2 * M_PI * (double)x[i])));
  }
  std::printf("revolutions in [0, 1): max |sin err| %.2e, max |cos err| %.2e\n", ws, wc);
  for (int i = 0; i < n; ++i) x[i] = (float)std::pow(10.0, -37.0 + 36.7 * i / (n - 1)) * ((i & 1) ? -1.f : 1.f);
  run();
  for (int dd = -37; dd < 0; dd += 3) {
    double w = 0;
    for (int i = 0; i < n; ++i) {
      const double ax = std::fabs((double)x[i]);
      if (ax < std::pow(10.0, dd) || ax >= std::pow(10.0, dd + 3)) continue;
      const double r = std::sin(2 * M_PI * (double)x[i]);
      w = std::fmax(w, std::fabs(s[i] - r) / std::fabs(r));
    }
    std::printf("small arguments 1e%d..1e%d rev: max rel sin err %.2e\n", dd, dd + 3, w);
  }
  (void)hipFree(dx);
  (void)hipFree(ds);
  (void)hipFree(dc);
  (void)hipFree(de);
  return 0;
}
