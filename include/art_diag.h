/*
 * art_diag.h -- measurements behind design decisions of libart (not part of
 * the transfer itself).
 *
 * art_diag_release_cost: the cost of making one workgroup's stores visible to
 * workgroups on other XCDs, the price a persistent, dependency-driven form of
 * the block-wavefront sweep (Sect. 3.1, 3.3) would pay per (block, bucket)
 * item.  A kernel of nwg one-wave workgroups each stores `words` floats and
 * then does nothing (mode 0), a device-scope fence (1), an agent-scope
 * release store of a flag (2), a relaxed store of a flag (3) or an
 * agent-scope acquire load of a flag (4); ns[mode] receives the best of five
 * timed launches (after one warm-up) divided by nwg, in nanoseconds per
 * workgroup.  nwg in [1, 1e6], words in [1, 65536]; allocates and frees its
 * own buffers and synchronises the device.  ART_E_INVAL for bad sizes.
 */
#ifndef ART_DIAG_H
#define ART_DIAG_H

#include "art.h"

#ifdef __cplusplus
extern "C" {
#endif

int art_diag_release_cost(int nwg, int words, float ns[5]);

#ifdef __cplusplus
}
#endif

#endif /* ART_DIAG_H */
