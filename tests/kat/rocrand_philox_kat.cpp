// Known-answer source for Philox4x32-10: prints the words of rocRAND's own
// (independent) implementation, run on the host through its public device/host
// API.  Usage: rocrand_philox_kat SEED SUBSEQUENCE OFFSET NBLOCKS
// Each output line is one 4-word block in hex.  rocrand_init(seed, subsequence,
// offset) starts the 128-bit counter at (offset/4 low 64 bits, subsequence high
// 64 bits) under key (seed low 32, seed high 32); every rocrand4() call returns
// one block and advances the counter's low 64 bits by one.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  unsigned long long seed = strtoull(argv[1], nullptr, 0);
  unsigned long long subsequence = strtoull(argv[2], nullptr, 0);
  unsigned long long offset = strtoull(argv[3], nullptr, 0);
  int nblocks = atoi(argv[4]);
  rocrand_state_philox4x32_10 state;
  rocrand_init(seed, subsequence, offset, &state);
  for (int i = 0; i < nblocks; ++i) {
    uint4 r = rocrand4(&state);
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
