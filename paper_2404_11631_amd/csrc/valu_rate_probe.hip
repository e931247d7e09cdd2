// valu_rate_probe.hip -- issue rate of single VALU instructions on gfx950 (and of the FP64 matrix
// instruction): 8 independent chains per lane, 8 waves per SIMD, timed with HIP events. Supports the
// ALU roofline of the path kernels (the per-normal instruction mix weighted by these rates gives the
// kernel's issue ceiling) and the matrix-core ceiling of the SQN product kernel.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#define CH 8
#define ITER 4096
#define BODY(ASM) \
  _Pragma("unroll 1") for (int it = 0; it < ITER; ++it) { \
    _Pragma("unroll") for (int c = 0; c < CH; ++c) { ASM; } }
__global__ void k_add(uint32_t* o, uint32_t s){ uint32_t a[CH]; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c+s;
  BODY(asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[c]) : "v"(s)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=a[c]; o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_xor3(uint32_t* o, uint32_t s){ uint32_t a[CH]; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c+s;
  BODY(asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[c]) : "v"(s)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=a[c]; o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_fma(uint32_t* o, uint32_t s){ float a[CH]; float x=__uint_as_float(s); for(int c=0;c<CH;++c)a[c]=threadIdx.x+c;
  BODY(asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(a[c]) : "v"(x)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=__float_as_uint(a[c]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_mad64(uint32_t* o, uint32_t s){ uint64_t a[CH]; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c+s;
  BODY(asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(a[c]) : "v"(s), "v"(s+1u) : "vcc"));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=(uint32_t)a[c]^(uint32_t)(a[c]>>32); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_mulhi(uint32_t* o, uint32_t s){ uint32_t a[CH]; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c+s;
  BODY(asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[c]) : "v"(s)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=a[c]; o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_mullo(uint32_t* o, uint32_t s){ uint32_t a[CH]; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c+s;
  BODY(asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[c]) : "v"(s)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=a[c]; o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_log(uint32_t* o, uint32_t s){ float a[CH]; for(int c=0;c<CH;++c)a[c]=1.5f+threadIdx.x+c;
  BODY(asm volatile("v_log_f32 %0, %0" : "+v"(a[c])));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=__float_as_uint(a[c]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_sin(uint32_t* o, uint32_t s){ float a[CH]; for(int c=0;c<CH;++c)a[c]=0.1f*c;
  BODY(asm volatile("v_sin_f32 %0, %0" : "+v"(a[c])));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=__float_as_uint(a[c]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_sqrt(uint32_t* o, uint32_t s){ float a[CH]; for(int c=0;c<CH;++c)a[c]=2.0f+c;
  BODY(asm volatile("v_sqrt_f32 %0, %0" : "+v"(a[c])));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=__float_as_uint(a[c]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
__global__ void k_fma64(uint32_t* o, uint32_t s){ double a[CH]; double x=1.0+s*1e-9; for(int c=0;c<CH;++c)a[c]=threadIdx.x+c;
  BODY(asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(a[c]) : "v"(x)));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=(uint32_t)__double_as_longlong(a[c]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
// FP64 matrix rate: 8 independent accumulators per wavefront of v_mfma_f64_16x16x4f64 (2,048 flops each)
typedef double f64x4 __attribute__((ext_vector_type(4)));
__global__ void k_mfma64(uint32_t* o, uint32_t s){ f64x4 acc[CH]; for(int c=0;c<CH;++c) acc[c]=f64x4{0.0,0.0,0.0,0.0};
  const double x=1.0+s*1e-9+threadIdx.x*1e-12, y=1.0-threadIdx.x*1e-12;
  BODY(acc[c]=__builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[c], 0, 0, 0));
  uint32_t r=0; for(int c=0;c<CH;++c) r^=(uint32_t)__double_as_longlong(acc[c][0]+acc[c][3]); o[blockIdx.x*blockDim.x+threadIdx.x]=r; }
typedef void(*K)(uint32_t*,uint32_t);
#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("%s: %s\n", #x, hipGetErrorString(e_)); return 1; } } while (0)
int main(){
  const int blocks = 256*4*8, threads = 256;   // 8 waves per SIMD worth
  uint32_t* o; CHECK(hipMalloc(&o, sizeof(uint32_t)*blocks*threads));
  struct {const char* n; K k;} ks[] = {{"v_add_u32",k_add},{"v_xor_b32",k_xor3},{"v_fma_f32",k_fma},{"v_mad_u64_u32",k_mad64},
    {"v_mul_hi_u32",k_mulhi},{"v_mul_lo_u32",k_mullo},{"v_log_f32",k_log},{"v_sin_f32",k_sin},{"v_sqrt_f32",k_sqrt},{"v_fma_f64",k_fma64}};
  hipEvent_t a,b; CHECK(hipEventCreate(&a)); CHECK(hipEventCreate(&b));
  for (auto& e : ks) {
    hipLaunchKernelGGL(e.k, dim3(blocks), dim3(threads), 0, 0, o, 3u);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a)); hipLaunchKernelGGL(e.k, dim3(blocks), dim3(threads), 0, 0, o, 3u); CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b)); float ms; CHECK(hipEventElapsedTime(&ms, a, b));
    double ops = (double)blocks*threads*ITER*CH;
    printf("%-16s %8.3f ms  %8.3f Tlane-ops/s\n", e.n, ms, ops/(ms*1e-3)/1e12);
  }
  {
    hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(threads), 0, 0, o, 3u);
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a)); hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(threads), 0, 0, o, 3u); CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b)); float ms; CHECK(hipEventElapsedTime(&ms, a, b));
    double flops = (double)blocks*(threads/64)*ITER*CH*2048.0;
    printf("%-16s %8.3f ms  %8.3f TFLOP/s\n", "v_mfma_f64_16x16x4f64", ms, flops/(ms*1e-3)/1e12);
  }
  hipError_t err = hipGetLastError(); printf("status %s\n", hipGetErrorString(err));
  CHECK(hipFree(o));
  return err == hipSuccess ? 0 : 1;
}
