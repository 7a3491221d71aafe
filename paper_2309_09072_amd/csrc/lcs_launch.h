// Host-side launchers of the single-pair kernels (defined in lcs_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcs_geom.h"

namespace lcs {

hipError_t launch_clear(int32_t *words, int32_t count, hipStream_t s);
hipError_t launch_nextmatch(const uint8_t *b, int32_t n, int32_t sigma, int32_t *nm, int32_t *err,
                            hipStream_t s);
hipError_t launch_base(int32_t h0, const uint8_t *a, int32_t n, int32_t sigma, const int32_t *nm,
                       int32_t *base0, int32_t *last, int32_t nstrips, int32_t hlast, int32_t *err,
                       hipStream_t s);
hipError_t launch_base_comb(int32_t h0, const uint8_t *a, const uint8_t *b, int32_t n,
                            int32_t sigma, int32_t *base0, int32_t *last, int32_t nstrips,
                            int32_t hlast, int32_t *comb, int32_t comb_stride, int32_t *rec,
                            int32_t *err, hipStream_t s);
hipError_t launch_anchor(const CombineArgs &c, int32_t npairs, hipStream_t s);
hipError_t launch_bracket(const CombineArgs &c, int32_t npairs, hipStream_t s);
hipError_t launch_length(const int32_t *top, int32_t m, int32_t n, int32_t *hdr, int4 *root,
                         hipStream_t s);
hipError_t launch_trace_splits(const TraceSplitArgs &t, hipStream_t s);
hipError_t launch_trace_leaf(int32_t h0, const uint8_t *a, int32_t n, int32_t sigma,
                             const int32_t *nm, int32_t nstrips, int32_t hlast, const int4 *nodes,
                             int32_t *a_idx, int32_t *b_idx, int32_t wcap, int32_t *err,
                             uint8_t *leaf, int64_t leaf_stride, hipStream_t s);
hipError_t launch_copy_len(const int32_t *hdr, int32_t *dst, hipStream_t s);
hipError_t launch_path(const int32_t *a_idx, const int32_t *b_idx, const int32_t *length,
                       int32_t cap, int32_t m, int32_t n, int32_t *col_in, int32_t *col_out,
                       hipStream_t s);
hipError_t launch_reverse(const uint8_t *src, int32_t len, uint8_t *dst, hipStream_t s);
hipError_t launch_unflip(const int32_t *hdr, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                         int32_t m, int32_t n, hipStream_t s);
hipError_t launch_semilocal(const int32_t *top, int32_t m, int32_t n, const int32_t *qi,
                            const int32_t *qk, int32_t count, int32_t *out, hipStream_t s);

}  // namespace lcs
