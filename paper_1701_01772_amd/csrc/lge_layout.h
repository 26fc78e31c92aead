// Sizes and layouts shared by the device code, the host runtime and the
// host-only arithmetic.  No HIP types: the host-only part also builds with a
// plain C++ compiler (the sanitizer build of the tests).
#pragma once

#include <stdint.h>

namespace lge {

// Number of 128-bit accumulators per estimate slot:
//   [0..12]  C3, C4, C5, C7, C8, C9, C10, C11, C12, C13, C14, C15, C16
//   [13..27] Q3 .. Q17 (sums of squared per-edge numerators 12*Y_i(e))
//   [28]     sampled edges
//   [29]     4-byte words read by the counting kernels
constexpr int kNumC = 13;
constexpr int kNumQ = 15;
constexpr int kAccIdxCount = 28;
constexpr int kAccIdxWords = 29;
constexpr int kAccSlots = 32;  // padded; one slot = 32 x (lo, hi) u64 = 512 B

// Edges whose endpoints both have degree <= kHubDeg are counted from LDS
// tables by one workgroup; the others are split across workgroups.
constexpr int kHubDeg = 1024;
// Vertices of degree > kHashDeg get a global hash table of their neighbours
// ("hub table"): O(1) membership tests instead of binary searches.
constexpr int kHashDeg = 32;
// The split kernel copies an endpoint's neighbours into an LDS table when its
// degree is <= kTableDeg and probes the endpoint's hub table otherwise.
constexpr int kTableDeg = 256;
// Ranked (co-degree table) vertices at most (rank + 1 fills 17 bits of the
// packed per-arc word), and the 64-bit words of one adjacency bit row over
// them.
constexpr int kMaxRanked = 131008;
// Co-degree rows hold one byte per vertex when no unranked vertex has degree
// above kRowMaxDeg (no co-degree with an unranked vertex can exceed it), else
// two.
constexpr int kRowMaxDeg = 254;
// At most this many co-degree rows (a row index fits 14 bits of a vertex's
// packed rank / row word).
constexpr int kMaxRows = 16383;
constexpr int kBitsWords = kMaxRanked / 64;
// Largest number of Gamma(a) positions handled by one global-class work item.
constexpr int kGlobalChunkMax = 1024;
// Vertex ids must stay below 2^29: the kernels keep three tag bits above them.
constexpr int64_t kMaxVertices = (int64_t)1 << 29;

}  // namespace lge
