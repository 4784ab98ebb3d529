// Declarations shared between the kernel translation units and the C-ABI
// layer (host side only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcad {

// bytes reserved for the per-launch control block at the start of a workspace
constexpr size_t kCtlBytes = 256;

// PCAD_OK for hipSuccess; otherwise records the error (pcad_last_hip_error)
// and returns PCAD_E_HIP
int hip_status(hipError_t e);

// tuning knobs (knobs.hip)
int knob_scan_threads(int op, int dir);  // dir 0 forward, 1 adjoint
int64_t knob_rbi_lds_max_bins(bool u64);
int64_t knob_rbi_elems_per_block();
int64_t knob_rbi_sort_min_bins();
bool knob_rbi_partition();
bool knob_rbi_parts();
int64_t knob_seg_tile();
int knob_seg_threads(int dir);

// stable sort of element indices by bin (sort.hip): keys outside [0, m)
// sort last as m
int sort_passes(int64_t m);
bool sort_supported(int64_t n);
size_t sort_ws_bytes(int64_t n, int64_t m);
hipError_t sort_by_key(const int32_t *keys, int64_t n, int64_t m, int32_t *keys_out,
                       int32_t *perm_out, void *ws, hipStream_t s);

// exclusive scan of ne uint32 entries in place (sort.hip); tot: scratch of
// iscan_totals(ne) entries, left zero; needs iscan_fits(ne)
int64_t iscan_totals(int64_t ne);
bool iscan_fits(int64_t ne);
hipError_t iscan_u32(uint32_t *v, int64_t ne, uint32_t *tot, hipStream_t s);

// partitioned reduce-by-index of one row for + * min max sumOfProd beyond the LDS
// histogram capacity (rbi_part.hip): `region` is the row's workspace part;
// writes every bin and the saved state (n0/ypos, argk, ssum) directly
bool rbi_part_may(int op, int64_t m);
size_t rbi_part_ws_bytes(int op, int64_t n, int64_t m);
hipError_t rbi_part_fwd_row(int op, int64_t n, int64_t m, const int32_t *idx, const float *v,
                            float *hist, uint32_t *n0, float *ypos, int32_t *argk, float *ssum,
                            void *region, hipStream_t s);

// sort-based reduce-by-index of one row (rbi_sorted.hip): `ctl` is the
// control block at the start of the call's workspace, `region` the row's
// workspace part (look-back status words; an accumulating ordered adjoint's
// L), `area` the row's part of the saved state (sorted keys, permutation and
// the sort's scratch)
size_t rbi_sort_area_bytes(int64_t n, int64_t m);
size_t rbi_sorted_ws_bytes(int op, int64_t n, int64_t m);
hipError_t rbi_sorted_fwd_row(int op, int64_t n, int64_t m, const int32_t *idx, const float *v,
                              float *hist, uint32_t *n0, float *ypos, uint64_t *keys, void *ctl,
                              void *region, void *area, hipStream_t s);
hipError_t rbi_sorted_vjp_row(int op, int64_t n, int64_t m, const float *v, const float *hbar,
                              float *vbar, bool accumulate, void *ctl, void *region,
                              const void *area, hipStream_t s);

// vectorised operators (vec.hip): transposes around the batched kernels;
// comb 0 reduce, 1 scan, 2 reduce-by-index
hipError_t transpose_launch(const float *in, float *out, int64_t batch, int64_t rows, int64_t cols,
                            bool accumulate, hipStream_t s);
size_t vec_tmp_bytes(int comb, int64_t batch, int64_t n, int64_t d, int64_t m);
hipError_t vreduce_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                              float *y, void *saved, void *ws, void *tmp, hipStream_t s);
hipError_t vreduce_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                              const void *saved, const float *ybar, float *xbar, bool accumulate,
                              void *ws, void *tmp, hipStream_t s);
hipError_t vscan_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                            void *saved, void *ws, void *tmp, hipStream_t s);
hipError_t vscan_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                            const void *saved, const float *ybar, float *xbar, bool accumulate,
                            void *ws, void *tmp, hipStream_t s);
hipError_t vrbi_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                           const int32_t *idx, const float *v, float *hist, void *saved, void *ws,
                           void *tmp, hipStream_t s);
hipError_t vrbi_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                           const int32_t *idx, const float *v, const void *saved,
                           const float *hbar, float *vbar, bool accumulate, void *ws, void *tmp,
                           hipStream_t s);

// d x d matrix-product scans, d = 3 or 5 (matd.hip)
int64_t matd_tiles(int d, int64_t batch, int64_t n);
size_t matd_saved_bytes(int d, int64_t batch, int64_t n);
size_t matd_ws_bytes(int d, int64_t batch, int64_t n);
hipError_t matd_fwd_launch(int d, int64_t batch, int64_t n, const float *x, float *y,
                           float *saved, void *ws, hipStream_t s);
hipError_t matd_vjp_launch(int d, int64_t batch, int64_t n, const float *x, const float *saved,
                           const float *ybar, float *xbar, bool accumulate, void *ws,
                           hipStream_t s);
hipError_t matd_reduce_fwd_launch(int d, int64_t batch, int64_t n, const float *x, float *y,
                                  float *saved, void *ws, hipStream_t s);
hipError_t matd_reduce_vjp_launch(int d, int64_t batch, int64_t n, const float *x,
                                  const float *saved, const float *ybar, float *xbar,
                                  bool accumulate, void *ws, hipStream_t s);

// block-diagonal matrix-product scans (bds.hip): k blocks of q x q, q in
// {1, 2, 3, 5}, k*q*q <= kBdsMaxBlockFloats; dir 0 forward, 1 adjoint
constexpr int64_t kBdsMaxBlockFloats = 4096;
bool bds_supported(int q, int64_t k);
size_t bds_tmp_bytes(int dir, int q, int64_t k, int64_t batch, int64_t n);
hipError_t bds_fwd_launch(int q, int64_t k, int64_t batch, int64_t n, const float *M, float *P,
                          void *saved, void *ws, void *tmp, hipStream_t s);
hipError_t bds_vjp_launch(int q, int64_t k, int64_t batch, int64_t n, const float *M,
                          const void *saved, const float *Pbar, float *Mbar, bool accumulate,
                          void *ws, void *tmp, hipStream_t s);

// int32 forward combinators for + * min max (i32.hip); comb 0 reduce, 1 scan,
// 2 reduce-by-index
size_t i32_ws_bytes(int comb, int64_t batch, int64_t n);
// tiles of an int32 scan over batch rows of n (one block each), at most
// kI32MaxScanTiles
int64_t i32_scan_tiles(int64_t batch, int64_t n);
constexpr int64_t kI32MaxScanTiles = (1LL << 24) - 1;
hipError_t i32_fwd_launch(int comb, int op, int64_t batch, int64_t n, int64_t m,
                          const int32_t *idx, const int32_t *x, int32_t *y, void *ws,
                          hipStream_t s);

// scan
int scan_tile_size(int op);
int scan_elem_floats(int op);
int scan_status_words(int op, bool abar);
hipError_t scan_fwd_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                           float *y0, float *y1, float *saved, float *total, bool reduce,
                           void *ws, hipStream_t s);
// tp0 (tp1): forward outputs y (LINREC: and A) for the checkpoint form,
// NULL for the recompute form, which reads `saved`
hipError_t scan_vjp_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                           const float *saved, const float *tp0, const float *tp1,
                           const float *yb0, const float *yb1, float *xb0, float *xb1,
                           bool accumulate, void *ws, hipStream_t s);

// reduce
int reduce_blocks_per_row(int64_t batch, int64_t n);
size_t reduce_ws_bytes(int op, int64_t batch, int64_t n);
hipError_t reduce_fwd_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             float *y, void *saved, void *ws, hipStream_t s);
hipError_t reduce_vjp_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             const void *saved, const float *ybar, float *xb0, float *xb1,
                             bool accumulate, void *ws, hipStream_t s);

// reduce-by-index
size_t rbi_ws_bytes(int op, int64_t batch, int64_t n, int64_t m);
size_t rbi_saved_bytes(int op, int64_t batch, int64_t n, int64_t m);
hipError_t rbi_fwd_launch(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                          const float *v, float *hist, void *saved, void *ws, hipStream_t s);
hipError_t rbi_vjp_launch(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                          const float *v, const void *saved, const float *hbar, float *vbar,
                          bool accumulate, void *ws, hipStream_t s);

}  // namespace pcad
