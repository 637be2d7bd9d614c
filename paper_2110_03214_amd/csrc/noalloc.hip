// Allocation-free form of the device-pointer batch (mapa_query_batch_noalloc).
//
// The batch pipeline needs a workspace beyond the caller's queries and
// results: per-query plans and (count, best) accumulators, the per-batch
// counters and the prefix work-list.  mapa_query_batch takes it from memory
// the context allocates and grows on demand; this entry point takes it from
// one file-scope device array instead, so a call issues kernel launches and
// stream/event operations only and never allocates or frees memory.  Each
// device the library runs on holds its own copy of the array until the
// process ends.  The kernels and the launch sequence are mapa_query_batch's.
#include <mutex>

#include "ctx.h"

namespace mapa {

namespace {

constexpr size_t kScratchBytes = (size_t)MAPA_NOALLOC_SCRATCH_MIB << 20;

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kOffPlan = 0;
constexpr size_t kOffCount = align256(kOffPlan + sizeof(Plan) * MAPA_NOALLOC_MAX_QUERIES);
constexpr size_t kOffBest = align256(kOffCount + sizeof(unsigned long long) * MAPA_NOALLOC_MAX_QUERIES);
constexpr size_t kOffCtr = align256(kOffBest + sizeof(unsigned long long) * MAPA_NOALLOC_MAX_QUERIES);
constexpr size_t kOffItems = align256(kOffCtr + sizeof(Counters));
constexpr unsigned long long kScratchItems = (kScratchBytes - kOffItems) / sizeof(uint2);
static_assert(kOffItems < kScratchBytes, "scratch too small for its fixed part");
static_assert(kScratchItems >= (unsigned long long)MAPA_NOALLOC_MAX_QUERIES + kPadReserve,
              "work-list part must hold the largest batch's padding");

// The workspace of every mapa_query_batch_noalloc call on this device.  In
// host code this name is a stand-in, not a device address: host code uses
// only the address hipGetSymbolAddress returns for it (g_scratch).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

// Zero n 8-byte words (the counters must start each batch at zero).
__global__ __launch_bounds__(256) void k_noalloc_clear(unsigned long long *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Resolve this device's copy of `scratch`; the device must be current.  Run
// once per device, from context creation.
int32_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(MAPA_ERR_UNSUPPORTED, "device %d: the allocation-free batch supports devices 0..%d",
                device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return MAPA_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(MAPA_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                hipGetErrorString(e));
  g_scratch[device] = static_cast<unsigned char *>(p);
  return MAPA_OK;
}

}  // namespace mapa

extern "C" int32_t mapa_query_batch_noalloc(mapa_ctx *c, const mapa_query *q, int32_t nq,
                                            mapa_result *res, void *stream) {
  using namespace mapa;
  if (!c) return fail(MAPA_ERR_INVALID_ARG, "ctx is NULL");
  if (c->serve) return fail(MAPA_ERR_STATE, "mapa_query_batch_noalloc: the serving loop owns the context");
  if (nq < 0) return fail(MAPA_ERR_INVALID_ARG, "nq < 0");
  if (nq > MAPA_NOALLOC_MAX_QUERIES)
    return fail(MAPA_ERR_ADMISSION, "batch of %d queries exceeds the allocation-free limit of %d",
                nq, MAPA_NOALLOC_MAX_QUERIES);
  if (nq == 0) return MAPA_OK;
  if (!q || !res) return fail(MAPA_ERR_INVALID_ARG, "NULL array");
  if (!c->has_device) return fail(MAPA_ERR_NO_DEVICE, "context has no device");
  if (c->server_topo.empty()) return fail(MAPA_ERR_UNKNOWN_SERVER, "no servers created");
  unsigned char *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = c->device < kMaxDevices ? g_scratch[c->device] : nullptr;
  }
  if (!base) return fail(MAPA_ERR_STATE, "scratch of device %d was not set up", c->device);
  MAPA_HIPCHK(hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace w;  // views into the scratch array; owns nothing
  w.cap_q = MAPA_NOALLOC_MAX_QUERIES;
  w.d_plan = reinterpret_cast<Plan *>(base + kOffPlan);
  w.d_acc_count = reinterpret_cast<unsigned long long *>(base + kOffCount);
  w.d_acc_best = reinterpret_cast<unsigned long long *>(base + kOffBest);
  w.d_ctr = reinterpret_cast<Counters *>(base + kOffCtr);
  w.d_items = reinterpret_cast<uint2 *>(base + kOffItems);
  w.cap_items = kScratchItems;
  MAPA_HIPCHK(hipStreamWaitEvent(s, c->last, 0));
  // the array keeps the previous call's contents: clear the counters (plans
  // and accumulators are written by the batch's first kernel)
  static_assert(sizeof(Counters) % sizeof(unsigned long long) == 0, "Counters size");
  const size_t words = sizeof(Counters) / sizeof(unsigned long long);
  hipLaunchKernelGGL(k_noalloc_clear, dim3(64), dim3(256), 0, s,
                     reinterpret_cast<unsigned long long *>(w.d_ctr), words);
  MAPA_HIPCHK(hipGetLastError());
  if (int32_t rc = enqueue_batch(c, w, q, res, nq, s)) return rc;
  MAPA_HIPCHK(hipEventRecord(c->last, s));
  ++c->batches;
  return MAPA_OK;
}
