// Device-wide exclusive scan and stable radix sort of (key, value) pairs, used
// by the tree build (sorting particles by leaf, leaf starts from leaf counts).
// Both are deterministic (no global atomics); buffers come from the caller.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tefmm {

// Scratch bytes needed by exclusive_scan for n elements.
size_t scan_scratch_bytes(int64_t n);
// out[i] = sum_{j < i} in[i] (unsigned 32-bit, wrapping), n <= 2^31 - 1; in and out may
// alias.  scratch: scan_scratch_bytes(n) bytes of device memory.
hipError_t exclusive_scan(const unsigned* in, unsigned* out, int64_t n, void* scratch, hipStream_t s);

// Scratch bytes needed by radix_sort_pairs for n elements.
size_t sort_scratch_bytes(int64_t n);
// Stable sort of (keys_in, vals_in) by the key bits [0, end_bit) into (keys_out,
// vals_out); n <= 2^31 - 1, end_bit <= 32.  The inputs are overwritten (they serve as
// the ping-pong buffers).  scratch: sort_scratch_bytes(n) bytes of device memory.
hipError_t radix_sort_pairs(unsigned* keys_in, unsigned* keys_out, int* vals_in, int* vals_out, int64_t n,
                            int end_bit, void* scratch, hipStream_t s);

}  // namespace tefmm
