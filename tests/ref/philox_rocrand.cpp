// External reference for the oracle's Philox4x32-10: rocRAND's header-only
// engine (an implementation independent of this repository).  Reads
// (counter[4], key[2]) as little-endian uint32 records from stdin and writes
// the four output words of each block to stdout.  Test infrastructure only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

namespace {
// the ten-round block function is a protected member of the engine
struct Block : rocrand_device::philox4x32_10_engine {
  uint4 run(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};
}  // namespace

int main() {
  Block b;
  uint32_t in[6];
  while (std::fread(in, sizeof(uint32_t), 6, stdin) == 6) {
    const uint4 r = b.run(uint4{in[0], in[1], in[2], in[3]}, uint2{in[4], in[5]});
    const uint32_t out[4] = {r.x, r.y, r.z, r.w};
    std::fwrite(out, sizeof(uint32_t), 4, stdout);
  }
  return 0;
}
