// Device memory whose streamed arrays lie far apart in physical memory.
//
// The fused step streams q direction arrays at once (one load and one store
// stream each).  On MI355X that access pattern runs at about 65 % of the HBM
// peak when the arrays are physically adjacent, as one allocation places
// them, and at 75-80 % once they are at least 3-4 GiB apart physically
// (measured with the kernel's own pattern; the spacing of the virtual
// addresses makes no difference).  This allocator cuts the buffer into
// pieces about one array long, creates each piece as its own physical
// allocation through the virtual memory API with a temporary spacer
// allocation after it, so that the next piece lands about SPREAD bytes
// further on, releases the spacers once every piece exists, and maps the
// pieces back to back into one virtual range.  The caller sees an ordinary
// contiguous buffer with the usual layout; the memory held is the buffer's
// own size (rounded up to whole pieces).  Spacers that cannot be made (too
// little free memory) are skipped: the buffer is then as correct, and
// possibly slower.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace lbmk {

namespace {

constexpr size_t SPREAD = (size_t)6 << 30;

struct Mapping {
  size_t offset, bytes;
  hipMemGenericAllocationHandle_t handle;
};
struct SpreadBuffer {
  size_t reserved = 0;
  std::vector<Mapping> maps;
};

std::mutex g_mu;
std::map<void *, SpreadBuffer> g_buffers;

size_t round_up(size_t v, size_t g) { return (v + g - 1) / g * g; }

void release(void *base, SpreadBuffer &b) {
  for (const Mapping &m : b.maps) {
    (void)hipMemUnmap((char *)base + m.offset, m.bytes);
    (void)hipMemRelease(m.handle);
  }
  b.maps.clear();
  if (b.reserved) (void)hipMemAddressFree(base, b.reserved);
  b.reserved = 0;
}

}  // namespace

int spread_alloc(size_t bytes, size_t offset, size_t stride, int count, void **out, std::string &msg) {
  *out = nullptr;
  if (bytes == 0 || count < 0 || offset + (size_t)count * stride > bytes) {
    msg = "spread allocation: arrays outside the buffer";
    return LBM_EINVAL;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  int vmm = 0;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, dev);
  if (e != hipSuccess) {
    msg = std::string("spread allocation: ") + hipGetErrorString(e);
    return LBM_EHIP;
  }
  if (!vmm) {
    msg = "spread allocation: the device has no virtual memory management";
    return LBM_EINVAL;
  }
  hipMemAllocationProp prop = {};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = dev;
  size_t gran = 0;
  e = hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityRecommended);
  if (e != hipSuccess || gran == 0) {
    msg = "spread allocation: no allocation granularity";
    return LBM_EHIP;
  }
  // The buffer is cut into pieces of one size P, a multiple of 2 MiB close
  // to the array stride, so that each array lies (mostly) in a piece of its
  // own.  The runtime maps pieces of one size back to back in a reservation,
  // but refuses some sequences of differing sizes (a 32 MiB piece after
  // 54 MiB ones), so the tail of the buffer is a whole piece as well.
  // Arrays of SPREAD bytes or more are far enough apart in one allocation:
  // then the buffer is a single piece.
  gran = (size_t)2 << 20;
  const size_t P = (count > 1 && stride > 0 && round_up(stride, gran) < SPREAD) ? round_up(stride, gran)
                                                                                 : round_up(bytes, gran);
  const size_t npieces = (bytes + P - 1) / P;
  const size_t total = npieces * P;
  std::vector<size_t> cut;
  for (size_t k = 0; k <= npieces; ++k) cut.push_back(k * P);
  SpreadBuffer buf;
  std::vector<hipMemGenericAllocationHandle_t> spacers;
  auto fail = [&](hipError_t err, const char *what) {
    for (hipMemGenericAllocationHandle_t s : spacers) (void)hipMemRelease(s);
    for (const Mapping &m : buf.maps) (void)hipMemRelease(m.handle);
    buf.maps.clear();
    msg = std::string("spread allocation: ") + what + ": " + hipGetErrorString(err);
    return err == hipErrorOutOfMemory || err == hipErrorMemoryAllocation ? LBM_ESIZE : LBM_EHIP;
  };
  for (size_t p = 0; p + 1 < cut.size(); ++p) {
    Mapping m{cut[p], cut[p + 1] - cut[p], {}};
    e = hipMemCreate(&m.handle, m.bytes, &prop, 0);
    if (e != hipSuccess) return fail(e, "hipMemCreate");
    buf.maps.push_back(m);
    // a spacer after each array piece pushes the next one further on
    if (m.bytes < SPREAD && p + 2 < cut.size()) {
      hipMemGenericAllocationHandle_t s;
      if (hipMemCreate(&s, round_up(SPREAD - m.bytes, gran), &prop, 0) == hipSuccess) spacers.push_back(s);
      else (void)hipGetLastError();
    }
  }
  for (hipMemGenericAllocationHandle_t s : spacers) (void)hipMemRelease(s);
  spacers.clear();
  void *base = nullptr;
  e = hipMemAddressReserve(&base, total, gran, nullptr, 0);
  if (e != hipSuccess) return fail(e, "hipMemAddressReserve");
  buf.reserved = total;
  hipMemAccessDesc acc = {};
  acc.location.type = hipMemLocationTypeDevice;
  acc.location.id = dev;
  acc.flags = hipMemAccessFlagsProtReadWrite;
  std::vector<Mapping> mapped;
  for (const Mapping &m : buf.maps) {
    e = hipMemMap((char *)base + m.offset, m.bytes, 0, m.handle, 0);
    if (e == hipSuccess) {
      mapped.push_back(m);
      e = hipMemSetAccess((char *)base + m.offset, m.bytes, &acc, 1);
    }
    if (e != hipSuccess) {
      for (const Mapping &u : mapped) (void)hipMemUnmap((char *)base + u.offset, u.bytes);
      (void)hipMemAddressFree(base, total);
      buf.reserved = 0;
      const std::string where = "hipMemMap of " + std::to_string(m.bytes) + " bytes at offset " +
                                std::to_string(m.offset) + " of a " + std::to_string(total) + "-byte range at " +
                                std::to_string((uintptr_t)base);
      return fail(e, where.c_str());
    }
  }
  std::lock_guard<std::mutex> lock(g_mu);
  g_buffers[base] = std::move(buf);
  *out = base;
  return LBM_OK;
}

int spread_free(void *ptr) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_buffers.find(ptr);
  if (it == g_buffers.end()) return LBM_EINVAL;
  // no kernel may still use the memory when it is unmapped
  (void)hipDeviceSynchronize();
  release(ptr, it->second);
  g_buffers.erase(it);
  return LBM_OK;
}

}  // namespace lbmk
