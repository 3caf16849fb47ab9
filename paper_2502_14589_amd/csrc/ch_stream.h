// Cache policy of the basis-column loads of the DCGS2 kernels.
#pragma once

#include <cstddef>

// Basis columns 0..k are read by the matvec and the update of DCGS2 iteration
// k and again by the next iteration.  Once they exceed the last-level cache
// (256 MB on this part) that cyclic scan gets no hits from it, and the column
// loads carry the streaming (non-temporal) hint so that they do not displace
// what is reused (the stencil halos, w, u).  Below that they keep the default
// policy and stay cached between iterations.
constexpr double CH_LLC_BYTES = 256.0 * 1024.0 * 1024.0;
inline bool stream_columns(size_t ldv, size_t esz, int k) { return double(ldv) * double(esz) * (k + 1) > CH_LLC_BYTES; }

// The 3-D matvec's w is read back by the update of the same iteration; in
// between, the two launches move about k + 3 columns (the basis, u, y and w).
// When those exceed the last-level cache, w does not survive there either, and
// it is written with the streaming hint, leaving the cache to the halos.
inline bool stream_store(size_t ldv, size_t esz, int k) { return double(ldv) * double(esz) * (k + 3) > CH_LLC_BYTES; }
