/*
 * motifs_testing.h -- test hooks of libmotifs.so (not for production use).
 *
 * They switch a prepared batch onto alternative internal paths whose
 * results must equal the default's, so that tests can compare them.
 */
#ifndef MOTIFS_TESTING_H
#define MOTIFS_TESTING_H

#include <stdint.h>

#include "motifs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Internal paths of the batch's later runs (0 restores the default):
   1 = every code straight to the histogram (no per-wave count hash),
   2 = flush the per-wave count hash after every insert,
   4 = MK_METHOD_CORES rescans every list instead of sharing a parent's arc
       pairs.
   Flags 1 and 2 switch the batch to builds of its counting kernel that
   carry these checks (the production builds leave them out).  The
   histograms are the same on every path. */
int mk_batch_debug(mk_batch *b, int32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* MOTIFS_TESTING_H */
