/*
 * cosenu_testing.h -- failure injection for the library's test-suite.
 * Not meant for applications: it exists so that the error paths of the C ABI
 * (exceptions turned into codes, a batch rebuild that fails half-way) can be
 * exercised from the host without faulting anything.
 */
#ifndef COSENU_TESTING_H
#define COSENU_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arms one failure at `site`, which fires the (after + 1)-th time the library
 * reaches that site and then disarms itself:
 *   1  parameter validation (cosenu_create, cosenu_batch_create) throws
 *      std::bad_alloc; the entry point must return COSENU_ENOMEM;
 *   2  parameter validation throws another C++ exception; the entry point
 *      must return COSENU_EDEVICE;
 *   3  a batch's task-list rebuild (creation, cosenu_batch_autotune) returns
 *      COSENU_EDEVICE; the batch must stay usable.
 * site 0 disarms.  Returns 0, or COSENU_EINVAL (-1) for an unknown site or a
 * negative `after`.  Process-wide; not thread-safe with concurrent calls. */
int cosenu_test_inject_failure(int32_t site, int32_t after);

#ifdef __cplusplus
}
#endif
#endif /* COSENU_TESTING_H */
