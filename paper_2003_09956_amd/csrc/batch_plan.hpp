// How the batched sweep cuts each system into work items and which row form
// it runs for the system: the host-side decisions that fix what the batched
// sweep kernel reads, kept apart from the rest of the batch host code.
#pragma once

#include <algorithm>
#include <cstdint>

namespace modap_host {

// Row-length bucket of a system whose rows take C 16-byte chunks per lane of
// a wavefront (C = 1, 2, 4, 8).
inline int bucket_of(int C) { return C == 1 ? 0 : C == 2 ? 1 : C == 4 ? 2 : 3; }

// Rows of one work item of a system: about cap_kib KiB of A, but a small
// system is still cut into min_items items of at least kMinItemKib KiB, so
// that a batch of few systems spreads over the device; a multiple of the
// wavefronts of a workgroup.  The partition depends on the system and the
// tile only, never on the other systems of the batch.  Eight items per system
// by default: a batch of few systems needs them to fill the device, while on
// a batch of many small systems every item costs a few microseconds of its
// own and fewer measure faster (the autotuner tries 1 to 16).
constexpr int64_t kMinItems = 8;
constexpr int64_t kMinItemKib = 32;
constexpr int32_t kMaxMinItems = 64;
inline int64_t plan_rows_per_item(int64_t m, int64_t ldA, int64_t elem_bytes, int32_t cap_kib, int32_t min_items,
                                  int64_t waves) {
    const int64_t sys_kib = m * ldA * elem_bytes / 1024;
    const int64_t cap = std::max<int32_t>(1, cap_kib);
    const int64_t least = min_items > 0 ? min_items : kMinItems;
    const int64_t kib = std::min(cap, std::max(kMinItemKib, sys_kib / least));
    int64_t r = kib * 1024 / (ldA * elem_bytes);
    r = std::max<int64_t>(waves, (r + waves - 1) / waves * waves);
    return std::min<int64_t>(r, (m + waves - 1) / waves * waves);
}

// Row form of a system: rows of at most 64 16-byte vectors (C == 1) run four
// to a wavefront, 16 lanes each, with 1, 2 or 4 chunks per lane; longer rows
// (or with the short form switched off) one to a wavefront with C chunks.
inline void plan_row_form(int64_t ldA, int64_t vec_elems, int C, bool short_form, int32_t *rpw, int32_t *chunks) {
    *rpw = 1;
    *chunks = C;
    if (C != 1 || !short_form) return;
    *rpw = 4;
    const int64_t per = 16 * vec_elems;
    const int64_t k = (ldA + per - 1) / per;
    *chunks = k <= 1 ? 1 : k <= 2 ? 2 : 4;
}

}  // namespace modap_host
