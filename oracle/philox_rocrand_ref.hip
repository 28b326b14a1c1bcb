// Independent Philox4x32-10 reference for pinning the oracle's generator.
// TEST INFRASTRUCTURE ONLY: built as a host-callable library from rocRAND's
// open-source device header; only tests/ load it.
#include <rocrand/rocrand_philox4x32_10.h>
#include <stdint.h>

namespace {
struct philox_probe : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
}  // namespace

extern "C" void ref_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox_probe p;
  uint4 c = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint2 k = {key[0], key[1]};
  uint4 o = p.block(c, k);
  out[0] = o.x; out[1] = o.y; out[2] = o.z; out[3] = o.w;
}
