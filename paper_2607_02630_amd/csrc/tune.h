// tune.h -- launch shapes chosen by the autotuner, read from a JSON cache.
//
// The cache (written by the package's autotune module) is found through the
// AESCTR_TUNE_CACHE environment variable, else as tune_cache.json beside the
// shared library.  Format:
//   {"entries": [{"variant": 1, "key_bits": 128, "size_log2": 23, "bpl": 2,
//                 "wg": 1024, "grid_per_cu": 1, "copies": 32, "tables": 2}, ...]}
// ("tables" may be absent: then 2 with 64 copies, 4 with 32; "first", the
// T-table kernel's first-chunk mode, may be absent: then the shape rule's.)
// The batch kernel's entry has "variant": 10 and carries "tiles_per_cu" and
// "max_tile_bytes" (the tile sizing rule's constants) and "bpl".
// A lookup takes the entry of the same variant and key size whose size_log2
// equals floor(log2(len)); a size the tuner did not time has no entry and
// keeps the built-in rule.
#pragma once

#include <stdint.h>

namespace aesctr {

struct TuneEntry {
    int variant = 0, key_bits = 0, size_log2 = 0;
    int bpl = 0, wg = 0, grid_per_cu = 0, copies = 0, tables = 0;
    int tiles_per_cu = 0, max_tile_bytes = 0;
    int first = -1;     // T-table first-chunk mode (Shape::wave_groups), -1 = not given
};

bool tune_lookup(int variant, int key_bits, uint64_t len, TuneEntry *out);

// Batch-kernel shape from the same cache (entries with "variant": 10).
bool tune_lookup_batch(TuneEntry *out);

}  // namespace aesctr
