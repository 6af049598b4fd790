// Host build of the register-resident DFTs of csrc/cmath.h, for the CPU tests:
// prints the input and dft<R, DIR> of a fixed sequence for R = 2 .. 32 and
// DIR = +1 (forward) and -1 (inverse, unnormalised).
#include <cmath>
#include <cstdio>

#include "cmath.h"

template <int R, int DIR>
static void run() {
  float2 v[R];
  for (int j = 0; j < R; ++j) {
    v[j] = make_float2(std::cos(0.37f * (float)(j * j) + 0.1f), std::sin(1.3f * (float)j) - 0.25f);
    std::printf("in %d %d %d %.9e %.9e\n", R, DIR, j, v[j].x, v[j].y);
  }
  mg::dft<R, DIR>(v);
  for (int j = 0; j < R; ++j) std::printf("out %d %d %d %.9e %.9e\n", R, DIR, j, v[j].x, v[j].y);
}

int main() {
  run<2, 1>(); run<4, 1>(); run<8, 1>(); run<16, 1>(); run<32, 1>();
  run<2, -1>(); run<4, -1>(); run<8, -1>(); run<16, -1>(); run<32, -1>();
  return 0;
}
