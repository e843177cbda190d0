// Host-side stand-ins for the HIP runtime calls the library makes, for
// replaying its host logic under AddressSanitizer on a machine without a GPU:
// device memory is host memory (so every upload, copy and fill is a checked
// memcpy/memset into the allocation it targets), streams, events and graphs
// are counters, kernel launches do nothing.  Results are meaningless; what is
// checked is that no host access leaves its allocation.  The kernel image
// symbol the host-only object references is supplied by the build (-D).
#define __HIP_PLATFORM_AMD__ 1
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>

extern "C" {
char HIP_FATBIN_SYMBOL[64] = {0};
static thread_local dim3 g_grid, g_block;
static thread_local size_t g_shm;
static thread_local hipStream_t g_st;
static std::atomic<long> g_launches{0};

static void* dev_alloc(size_t n) { return aligned_alloc(256, (n + 255) / 256 * 256 + 256); }
static int& obj(void* h) { return *static_cast<int*>(h); }

hipError_t hipMalloc(void** p, size_t n) { *p = dev_alloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = dev_alloc(n); return *p ? hipSuccess : hipErrorOutOfMemory; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemset(void* d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = reinterpret_cast<hipEvent_t>(new int(0)); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete &obj(e); return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t e) { (void)obj(e); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { ++obj(e); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { (void)obj(e); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = reinterpret_cast<hipStream_t>(new int(0)); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned int) { (void)obj(e); return hipSuccess; }
// Streams being captured: a capture begun on a stream that is already
// capturing (two host threads recording into one graph) aborts the replay.
static std::mutex g_cap_mu;
static std::set<hipStream_t>* g_capturing = new std::set<hipStream_t>;
static std::atomic<long> g_captures{0};
long hip_stub_captures(void) { return g_captures.load(); }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  ++g_captures;
  std::lock_guard<std::mutex> lk(g_cap_mu);
  if (!g_capturing->insert(s).second) {
    fprintf(stderr, "HIP stand-in: a capture began on a stream that is already capturing\n");
    abort();
  }
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  {
    std::lock_guard<std::mutex> lk(g_cap_mu);
    g_capturing->erase(s);
  }
  *g = reinterpret_cast<hipGraph_t>(new int(1));
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  (void)obj(g);
  *x = reinterpret_cast<hipGraphExec_t>(new int(2));
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { (void)obj(x); return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete &obj(g); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete &obj(x); return hipSuccess; }
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "HIP stand-in"; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipLaunchKernel(const void*, dim3, dim3, void**, size_t, hipStream_t) { ++g_launches; return hipSuccess; }
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t s, hipStream_t st) {
  g_grid = g; g_block = b; g_shm = s; g_st = st;
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* s, hipStream_t* st) {
  *g = g_grid; *b = g_block; *s = g_shm; *st = g_st;
  return hipSuccess;
}
void** __hipRegisterFatBinary(const void*) { static void* m = nullptr; return &m; }
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*, int*) {}
void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}
void __hipUnregisterFatBinary(void**) {}
long stub_kernel_launches(void) { return g_launches.load(); }
}
