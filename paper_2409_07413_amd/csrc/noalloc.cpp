// Allocation-free form of the unitary 2D FFT entry point, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// spr_fft2 takes its twiddle table from the context (built on the first call
// of a size) and transforms the rows into the output buffer.  This form keeps
// both the twiddle table and the row-transform intermediate in one
// file-scope device array, `scratch`, of kScratchBytes: each GPU holds its
// own copy from module load until the process ends.  Host code never uses
// the array's name as an address: the context creation call looks up the
// device address of the array on its device (hipGetSymbolAddress, with that
// device current) and keeps it per device; kernels receive that address as an
// argument.
//
// Every call on one GPU shares the array and leaves its contents behind;
// nothing in it has to start at zero (every call writes the twiddles and the
// intermediate it reads).  Calls that overlap on one GPU (different streams,
// or host threads racing on the same stream) race on the array.
#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch;  // device -> device address of its `scratch`

constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Twiddles exp(-2 pi i e / n) for e < n, in FP64 rounded once to float: the
// definition of the table the other entry points build on the host.
__global__ void k_twiddle_fill(float2* tw, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    double s, c;
    sincospi(2.0 * (double)e / (double)n, &s, &c);
    tw[e] = make_float2((float)c, (float)-s);
  }
}

}  // namespace

// Called by spr_ctx_create with the context's device current: the device
// address of this device's copy of `scratch`.
spr_status noalloc_setup(int device, std::string* err) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch.count(device)) return SPR_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return SPR_E_HIP;
  }
  g_scratch[device] = static_cast<unsigned char*>(p);
  return SPR_OK;
}

spr_status spr_fft2_noalloc(spr_ctx* ctx, int32_t n, int32_t batch, const float* in, float* out, int32_t inverse,
                            void* hip_stream) {
  if (!ctx || !in || !out || batch < 0) return SPR_E_INVALID_ARG;
  return guarded(ctx, [&] {
    const SizeKernels* K = ctx_kernels(ctx, n);
    if (!K) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported size " + std::to_string(n));
    if (batch == 0) return;
    const size_t tw_bytes = round256((size_t)n * sizeof(float2));
    const size_t need = tw_bytes + (size_t)batch * n * n * sizeof(float2);
    if (need > kScratchBytes)
      fail(SPR_E_INVALID_ARG, "spr_fft2_noalloc: " + std::to_string(batch) + " images of " + std::to_string(n) +
                                  "^2 need " + std::to_string(need) + " bytes of scratch, the maximum is " +
                                  std::to_string(kScratchBytes));
    unsigned char* base = nullptr;
    {
      std::lock_guard<std::mutex> g(g_scratch_mu);
      auto it = g_scratch.find(ctx->device);
      if (it != g_scratch.end()) base = it->second;
    }
    if (!base) fail(SPR_E_HIP, "spr_fft2_noalloc: the scratch address of this device was not set up");
    use_device(ctx);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    float2* tw = reinterpret_cast<float2*>(base);
    float2* mid = reinterpret_cast<float2*>(base + tw_bytes);
    hipLaunchKernelGGL(k_twiddle_fill, dim3((n + 255) / 256), dim3(256), 0, s, tw, n);
    launch_ok(hipGetLastError(), "twiddle_fill");
    const int dir = inverse ? +1 : -1;
    RowFftArgs r{nullptr, nullptr, batch, reinterpret_cast<const float2*>(in), mid, dir, 1.f, tw};
    launch_ok(K->row_fft(r, s), "row_fft");
    ColFftArgs c{nullptr, nullptr, batch, mid, reinterpret_cast<float2*>(out), dir, 1.f / (float)n, tw};
    launch_ok(K->col_fft(c, s), "col_fft");
  });
}
