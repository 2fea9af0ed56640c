// Shape of the LDS stage of the staged applies (host-visible constants, no device types, so
// that the limits they imply can be built and tested on their own).
//
// A workgroup of a staged apply owns a patch of kPatchRows x kPatchCols scan positions and
// keeps the input rows its current stage unit reads in LDS as a ring of kPatchRows + 1 slots.
// A slot holds the patch's columns plus a halo of k_half columns on each side; each column is
// one 64-byte chunk of the inner axis padded to kColumnBytes (the padding spreads the
// columns over the LDS banks).  The lateral model extent k_half is therefore limited by the
// LDS of one compute unit.
#pragma once

namespace aroam {

constexpr int kPatchRows = 8;        // scan rows per workgroup patch
constexpr int kPatchCols = 32;       // scan columns per workgroup patch (two 16-position tiles)
constexpr int kChunkBytes = 64;      // inner-axis entries of one staged column (bytes)
constexpr int kColumnBytes = 80;     // LDS stride of a staged column: chunk + 16 bytes of padding
constexpr long long kLdsBytes = 160 * 1024;  // LDS of one gfx950 compute unit

// LDS bytes of the row ring of a staged apply with offsets -k_half .. k_half.
constexpr long long staged_lds_bytes(int k_half) {
  return (long long)(kPatchRows + 1) * (kPatchCols + 2 * k_half) * kColumnBytes;
}

// Largest k_half whose row ring fits the LDS.
constexpr int max_k_half() {
  int k = 0;
  while (staged_lds_bytes(k + 1) <= kLdsBytes) ++k;
  return k;
}

}  // namespace aroam
