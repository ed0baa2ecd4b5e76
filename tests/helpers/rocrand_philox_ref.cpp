// Host-side known-answer generator: evaluates rocRAND's Philox4x32-10 round
// function (header-only, host-callable) on counters/keys read from stdin and
// prints the four output words.  Used only to pin the oracle's generator
// against an independent library implementation.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// The round function is a protected member; a derived class re-exports it.
struct Engine : rocrand_device::philox4x32_10_engine {
  using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Engine eng;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 ctr = {c0, c1, c2, c3};
    uint2 key = {k0, k1};
    uint4 r = eng.ten_rounds(ctr, key);
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
