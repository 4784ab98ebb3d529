// Tuning knobs: the launch parameters an autotuner may choose (block sizes of
// the scan kernels, the reduce-by-index strategy threshold and chunking).
// No knob changes a result's layout or a saved state's layout; only speed
// depends on them.  Values are process-wide and read at launch time.
#include <string.h>

#include "../../include/pcad.h"
#include "internal.hpp"

namespace pcad {
namespace {

struct Knob {
  const char *name;
  int64_t def, lo, hi;
  bool pow2;  // value must be a power of two
  int64_t value;
};

// order: scan forward threads by operator, scan adjoint threads by operator,
// then the reduce-by-index knobs (indices used below)
Knob g_knobs[] = {
    {"scan.fwd.threads.add", 1024, 256, 1024, true, 1024},
    {"scan.fwd.threads.mul", 1024, 256, 1024, true, 1024},
    {"scan.fwd.threads.min", 1024, 256, 1024, true, 1024},
    {"scan.fwd.threads.max", 1024, 256, 1024, true, 1024},
    {"scan.fwd.threads.linrec", 512, 256, 1024, true, 512},
    {"scan.fwd.threads.mat2", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.add", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.mul", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.min", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.max", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.linrec", 512, 256, 1024, true, 512},
    {"scan.vjp.threads.mat2", 512, 256, 1024, true, 512},
    // bins up to which a block keeps a private LDS histogram (+ and *: float
    // values; min/max: 64-bit keys); above it, global atomics
    {"rbi.lds_max_bins_f32", 8192, 0, 8192, false, 8192},
    {"rbi.lds_max_bins_u64", 4096, 0, 4096, false, 4096},
    // elements per block of the histogram kernels
    {"rbi.elems_per_block", 16384, 1024, 1 << 20, true, 16384},
    // beyond the LDS histogram, bin counts from which the commutative
    // operators sort by bin instead of combining in an LDS hash table (the
    // hash table measured faster at every bin count up to 2^22, uniform and
    // Zipf keys, so by default only the ordered operators sort)
    {"rbi.sort_min_bins", 1 << 26, 0, 1 << 26, false, 1 << 26},
    // beyond the LDS histogram: 1 partitions the elements by bin range and
    // builds LDS histograms per range, 0 uses the LDS hash table
    {"rbi.partition", 1, 0, 1, false, 1},
    // bin counts of at most four 128 KB LDS tables (+: 131072, min/max:
    // 65536), one row: 1 splits the bins into those tables, one block per
    // (table, chunk of elements); 0 leaves them to the partition / hash path
    {"rbi.parts", 1, 0, 1, false, 1},
    // batched segmented plans (read when a plan is created): elements per
    // work item, and the block sizes of the forward and adjoint kernels
    {"seg.tile", 8192, 4096, 8192, true, 8192},
    {"seg.fwd.threads", 512, 256, 1024, true, 512},
    {"seg.vjp.threads", 512, 256, 1024, true, 512},
};
constexpr int kNumKnobs = (int)(sizeof(g_knobs) / sizeof(g_knobs[0]));
constexpr int kRbiF32 = 12, kRbiU64 = 13, kRbiEpb = 14, kRbiSort = 15, kRbiPart = 16,
              kRbiParts = 17, kSegTile = 18, kSegFwdThreads = 19, kSegVjpThreads = 20;

Knob *find(const char *name) {
  if (!name) return nullptr;
  for (Knob &k : g_knobs)
    if (strcmp(k.name, name) == 0) return &k;
  return nullptr;
}

}  // namespace

// saturated addition has the shape of + and shares its block sizes;
// sumOfProd scans (two floats per element) share the linear recurrence's
int knob_scan_threads(int op, int dir) {
  const int o = op == PCAD_SATADD ? PCAD_ADD : (op == PCAD_SUMPROD ? PCAD_LINREC : op);
  return (int)g_knobs[(dir ? 6 : 0) + o].value;
}
int64_t knob_rbi_lds_max_bins(bool u64) { return g_knobs[u64 ? kRbiU64 : kRbiF32].value; }
int64_t knob_rbi_elems_per_block() { return g_knobs[kRbiEpb].value; }
int64_t knob_rbi_sort_min_bins() { return g_knobs[kRbiSort].value; }
bool knob_rbi_partition() { return g_knobs[kRbiPart].value != 0; }
bool knob_rbi_parts() { return g_knobs[kRbiParts].value != 0; }
int64_t knob_seg_tile() { return g_knobs[kSegTile].value; }
int knob_seg_threads(int dir) { return (int)g_knobs[dir ? kSegVjpThreads : kSegFwdThreads].value; }

}  // namespace pcad

using namespace pcad;

extern "C" {

int pcad_knob_count(void) { return kNumKnobs; }

const char *pcad_knob_name(int i) { return (i >= 0 && i < kNumKnobs) ? g_knobs[i].name : nullptr; }

int pcad_knob_get(const char *name, int64_t *value) {
  if (!name || !value) return PCAD_E_NULLPTR;
  const Knob *k = find(name);
  if (!k) return PCAD_E_INVALID_ARG;
  *value = k->value;
  return PCAD_OK;
}

int pcad_knob_set(const char *name, int64_t value) {
  if (!name) return PCAD_E_NULLPTR;
  Knob *k = find(name);
  if (!k) return PCAD_E_INVALID_ARG;
  if (value < k->lo || value > k->hi) return PCAD_E_INVALID_ARG;
  if (k->pow2 && (value & (value - 1)) != 0) return PCAD_E_INVALID_ARG;
  k->value = value;
  return PCAD_OK;
}

void pcad_knob_reset(void) {
  for (Knob &k : g_knobs) k.value = k.def;
}

}  // extern "C"
