/*
 * sv_util.h -- measurement utility exported by libsv.so beside the
 * simulator entry points of sv.h.
 *
 * sv_util_copy copies `bytes` (a multiple of 16) from device buffer `src` to
 * device buffer `dst` with the same access pattern the state sweeps use (16-byte
 * non-temporal loads and stores, 8 per lane).  It is the reference kernel for
 * the achievable HBM read+write bandwidth and for calibrating the memory
 * traffic counters against a kernel of known size.  Both buffers are owned by
 * the caller; they must not overlap.  Async on `hip_stream` (NULL = null
 * stream).  Returns SV_OK, SV_ERR_ARG (null pointer, size not a multiple of
 * 16) or SV_ERR_DEVICE.
 */
#ifndef SV_UTIL_H
#define SV_UTIL_H
#include <stddef.h>

#include "sv.h"

#ifdef __cplusplus
extern "C" {
#endif

sv_status sv_util_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SV_UTIL_H */
