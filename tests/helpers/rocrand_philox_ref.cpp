// Host-only reference: prints rocRAND's Philox4x32-10 output for given
// counters and keys.  Used by the oracle's Philox pin.  Runs no GPU code.
//
// Input lines:  c0 c1 c2 c3 k0 k1   (decimal uint32)
// Output lines: r0 r1 r2 r3         (decimal uint32)
//
// rocRAND's engine(seed, subsequence, offset) starts at counter
// (offset/4 lo, offset/4 hi, subsequence lo, subsequence hi) with key
// (seed lo, seed hi), so any counter/key pair can be reached.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = k0 | (k1 << 32);
    unsigned long long subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_state_philox4x32_10 st(seed, subseq, offset);
    uint4 r = st.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
