// Prints, for every slot of four 1,024-slot blocks, the word and bit the
// library's layout helpers give it in a posting-bitmap row and in the live
// bitmap. Built for the host by the CPU test suite; runs no GPU code.
#include <cstdio>

#include "snn_device.h"

int main() {
  for (unsigned s = 0; s < 4096; ++s)
    std::printf("%u %u %u %u %u\n", s, snn::post_word(s), snn::post_bit(s), snn::slot_word(s), snn::slot_bit(s));
  return 0;
}
