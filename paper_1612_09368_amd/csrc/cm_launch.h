// Host-side launch helpers of the kernels in cm_kernels.hip.
#pragma once
#include "cm_internal.h"

namespace cm {

hipError_t fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
hipError_t fill_u64(unsigned long long *p, unsigned long long v, int64_t n, hipStream_t st);
hipError_t fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t st);
hipError_t ctl_batch_reset(Ctl *c, int cur, hipStream_t st);
hipError_t ctl_reserve_reset(Ctl *c, hipStream_t st);
hipError_t ctl_set_pool(Ctl *c, unsigned long long tail, hipStream_t st);
hipError_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp,
                              int64_t *total_dev, hipStream_t st);
int64_t scan_tmp_len(int64_t n);

hipError_t load_check(const int32_t *src, const int32_t *dst, int64_t m, int32_t n,
                      unsigned long long *hkey, int64_t *hval, uint32_t mask,
                      unsigned long long *first_bad, hipStream_t st);
hipError_t count_deg(const int32_t *src, const int32_t *dst, int64_t m, int32_t *len, hipStream_t st);
hipError_t caps_from_counts(const int32_t *cnt, int32_t n, int32_t n_cap, int64_t *caps64,
                            int32_t *cap, hipStream_t st);
hipError_t scatter_edges(const int32_t *src, const int32_t *dst, int64_t m, const int64_t *off,
                         int32_t *len, int32_t *nbr, hipStream_t st);
hipError_t count_live(const KArgs &a, int32_t *cnt, int blocks, hipStream_t st);
hipError_t repack_copy(const KArgs &a, const int64_t *newoff, int32_t *newnbr, int blocks, hipStream_t st);
hipError_t repack_finish(const KArgs &a, const int64_t *newoff, const int32_t *cnt, int blocks,
                         hipStream_t st);
hipError_t export_edges(const KArgs &a, int32_t *xs, int32_t *ys, int64_t cap,
                        unsigned long long *tail, int blocks, hipStream_t st);

hipError_t dec_prep(const KArgs &a, int blocks, hipStream_t st);
hipError_t decompose_coop(const KArgs &a, int blocks, hipStream_t st);
hipError_t mcd_init(const KArgs &a, int blocks, hipStream_t st);

hipError_t validate_batch(const KArgs &a, int blocks, hipStream_t st);
hipError_t reserve_gain(const KArgs &a, int blocks, hipStream_t st);
hipError_t reserve_alloc_copy(const KArgs &a, int blocks, hipStream_t st);
hipError_t delete_compact(const KArgs &a, int blocks, hipStream_t st);
hipError_t maintain_coop(const KArgs &a, int blocks, hipStream_t st);
hipError_t program_coop(const KArgs &a, int blocks, hipStream_t st);
const void *program_kernel();
hipError_t serve_coop(const KArgs &a, int blocks, hipStream_t st);

hipError_t vins_init(const KArgs &a, int32_t first, int32_t c, hipStream_t st);
hipError_t vins_revert(const KArgs &a, int32_t first, int32_t c, hipStream_t st);
hipError_t vins_expand(const int64_t *off, int32_t c, int32_t first, int32_t *src, int blocks,
                       hipStream_t st);
hipError_t vins_check_off(const int64_t *off, int32_t c, unsigned long long *first_bad, hipStream_t st);
hipError_t vdel_check(const KArgs &a, const int32_t *ids, int32_t c, int32_t *firstidx,
                      unsigned long long *first_bad, unsigned long long *total, hipStream_t st);
hipError_t vdel_gather(const KArgs &a, const int32_t *ids, int32_t c, int32_t *xs, int32_t *ys,
                       int64_t cap, unsigned long long *tail, int blocks, hipStream_t st);
hipError_t vdel_finish(const KArgs &a, const int32_t *ids, int32_t c, hipStream_t st);

// which: 0 = maintenance kernel, 1 = decomposition kernel, 2 = batch program kernel
hipError_t coop_occupancy(int which, int *blocks_per_cu);

}  // namespace cm
