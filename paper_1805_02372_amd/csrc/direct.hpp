// Host entry points of the direct GF(2) path and the word XOR (direct.hip).
#pragma once
#include <stdint.h>

namespace pa {

// Reversed-key words the direct path needs for an n-bit key (scratch `kr`).
uint64_t direct_key_words(uint64_t n);
// Direct product of one job in two launches on `stream`: the prep kernel
// (reversed key into kr, direct_key_words(n) 32-bit words; out cleared), then
// the product kernels, which XOR each output bit into out (m bits).  Each
// returns 0, or -1 on a launch error, and adds its launches to *launches.
int launch_direct_prep(const uint64_t* key, uint64_t n, uint64_t m, uint64_t* out, uint32_t* kr, void* stream,
                       uint64_t* launches);
int launch_direct_main(const uint64_t* seed, uint64_t n, uint64_t m, uint64_t* out, const uint32_t* kr,
                       void* stream, uint64_t* launches);
// Selected outputs: bit k of res (ceil(count/64) words) = y[idx[k]].
int launch_direct_select(const uint64_t* seed, const uint64_t* key, uint64_t n, uint64_t m, const uint64_t* idx,
                         uint32_t count, uint64_t* res, uint32_t* kr, void* stream);
// dst[k] ^= src[k] for k < words (stream order); src may be dst (clears it).
int launch_xor_words(uint64_t* dst, const uint64_t* src, uint64_t words, void* stream);

}  // namespace pa
