/*
 * henn_testing.h -- test-only flags and entry points of libhenn.
 *
 * Not part of the stable interface of henn.h.  Test suites use them to reach
 * alternative code paths that must give results identical to the default
 * ones, and the error paths of the library.  Same conventions as henn.h.
 */
#ifndef HENN_TESTING_H
#define HENN_TESTING_H

#include "henn.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Search flags (henn_search_params.flags) that select an alternative path
 * with the same results: */
#define HENN_SEARCH_NO_ROOT_KERNEL 4u /* scan a complete-graph root inside the search
                                         kernel instead of a separate scan */
#define HENN_SEARCH_ROOT_VALU 8u      /* scan a complete-graph root with the tiled
                                         VALU kernel instead of the matrix-core
                                         shortlist + exact check */
#define HENN_SEARCH_VIS32 16u         /* keep full 32-bit ids in the visited table
                                         even where 8- or 16-bit tags are exact */
#define HENN_SEARCH_VIS16 32u         /* keep 16-bit tags where 8-bit tags would be
                                         exact */

/* Allocation-failure injector for the error paths.  n >= 0: the next n device
 * allocations of the library succeed and every later one fails as out of
 * memory (the calls return HENN_E_NOMEM, and release what they allocated)
 * until the injector is set again; n < 0 turns it off (the default).
 * Process-wide; counts the allocations of every thread. */
henn_status henn_testing_fail_alloc_after(int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* HENN_TESTING_H */
