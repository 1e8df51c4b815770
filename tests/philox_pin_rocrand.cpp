// Independent Philox4x32-10 pin: prints rocRAND's host-side philox4x32_10
// engine output for counters and keys read from stdin ("c0 c1 c2 c3 k0 k1" in
// hex per line).  rocRAND addresses the counter as (offset/4 -> words 0,1;
// subsequence -> words 2,3) and the key as the 64-bit seed, so any counter with
// word1 < 2^30 is reachable.  Host code only; nothing runs on a GPU.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
  return 0;
}
