// wv_internal.h -- declarations shared by the HIP translation units of
// libwavelet (not part of the C-ABI).
#pragma once

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "wv_common.h"

// ---- optional per-kernel timing (wv_profile.hip) ----------------------------
int wv_prof_before(hipStream_t s);
void wv_prof_after(int slot, hipStream_t s, const char* name);
// run `launch` (one or more kernel launches on stream s), bracketed by events
// named `name` when `on`
#define WV_TIMED(on, s, name, launch)                  \
    do {                                               \
        const int slot_ = (on) ? wv_prof_before(s) : -1; \
        launch;                                        \
        if (slot_ >= 0) wv_prof_after(slot_, s, name); \
    } while (0)

// ---- prefix sum (wv_scan.hip) ----------------------------------------------
// scratch entries (uint64) the scan of `count` items in `ncols` columns needs
uint64_t wv_scan_partials(uint64_t count, uint32_t ncols);
// exclusive prefix of in[i*ncols+c] into out[i*ncols+c]; totals[c] = sum
hipError_t wv_scan_u32(const uint32_t* in, uint64_t* out, uint64_t count, uint32_t ncols,
                       uint64_t* partial, uint64_t* totals, hipStream_t s);

// ---- directories (wv_directory.hip) ----------------------------------------
// Rank directory + sampled select of one binary level whose words are already
// written and whose per-superblock ones counts are in sb_ones.  Writes the
// level's zeros/ones into its descriptor and the zero count to *zl_dev.
struct wv_dir_scratch {
    uint32_t* sb_ones;   // ceil(n/512) counts (filled by the level writer)
    uint64_t* sb_pre;    // ceil(n/512)
    uint64_t* partial;   // wv_scan_partials(ceil(n/512), 1)
    uint64_t* total;     // 1 entry: ones on the level
};
hipError_t wv_binary_directory(uint8_t* image, uint32_t level, const wv_level& L,
                               const wv_dir_scratch& sc, uint64_t* zl_dev, hipStream_t s);
// ones per superblock of an already written binary level (when the level
// writer did not produce them)
hipError_t wv_count_superblocks(const uint8_t* image, const wv_level& L, uint32_t* sb_ones,
                                hipStream_t s);

// Directories of several binary levels (levels l0..l0+nl-1, sizes from the
// layout) with one launch per step: per-chunk ones counts, a column-wise
// prefix sum, then every chunk writes its superblocks and select samples.
// The sizes come from the longest level, n.
struct wv_span_dir {
    uint64_t nchunks, nl;
    uint64_t off_cnt, off_pre, off_part, off_tot, bytes;
};
wv_span_dir wv_span_dir_sizes(uint64_t n, uint32_t nl);
hipError_t wv_span_directory(uint8_t* image, const wv_layout_out& lay, uint32_t l0, uint32_t nl,
                             uint8_t* scratch, const wv_span_dir& sz, hipStream_t s, bool prof = false);

// per-digit counters of M multiary levels of the same length (from lv[0])
struct wv_mdir_scratch {
    uint32_t* rng_cnt;   // ranges * M * d
    uint64_t* rng_pre;   // ranges * M * d
    uint64_t* partial;   // wv_scan_partials(ranges, M * d)
    uint64_t* totals;    // M * d
};
hipError_t wv_multiary_counters(uint8_t* image, const wv_level* lv, uint32_t M, uint32_t D,
                                const wv_mdir_scratch& sc, hipStream_t s);
// the range counters alone, once sc.rng_cnt holds every range's digit counts
// and the sub-range counters are written (by the gather of the tree levels)
hipError_t wv_multiary_ranges(uint8_t* image, const wv_level* lv, uint32_t M, uint32_t D,
                              const wv_mdir_scratch& sc, hipStream_t s);

// ---- pinned host staging -------------------------------------------------------
// Pinned host buffers for copies a build issues between launches (the symbol
// counts a tree build reads back and the tables it uploads, the descriptors
// of a batch): a copy from or to pageable memory holds the host until it
// completes.  Buffers are reused
// until the process ends; one that a failed build may still be copying is
// not returned.
class PinnedBuf {
public:
    explicit PinnedBuf(size_t bytes)
    {
        if (!bytes) return;   // nothing to hold
        std::lock_guard<std::mutex> lk(mu());
        auto& fr = pool();
        for (size_t i = 0; i < fr.size(); i++)
            if (fr[i].second >= bytes) {
                p_ = fr[i].first;
                n_ = fr[i].second;
                fr.erase(fr.begin() + (long)i);
                return;
            }
        n_ = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&p_, n_, hipHostMallocDefault) != hipSuccess) p_ = nullptr;
    }
    ~PinnedBuf()
    {
        if (!p_ || !idle_) return;
        std::lock_guard<std::mutex> lk(mu());
        pool().push_back({p_, n_});
    }
    void* get() const { return p_; }
    void idle() { idle_ = true; }   // no copy into it is pending any more
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;

private:
    static std::mutex& mu()
    {
        static std::mutex m;
        return m;
    }
    static std::vector<std::pair<void*, size_t>>& pool()
    {
        static std::vector<std::pair<void*, size_t>> v;
        return v;
    }
    void* p_ = nullptr;
    size_t n_ = 0;
    bool idle_ = false;
};

// A second stream of the current device for work a build forks off its own
// stream and joins again with events (created on first use, default
// priority, never destroyed); nullptr when it cannot be created.
hipStream_t wv_side_stream();

// ---- header (wv_directory.hip) ---------------------------------------------
// header, level descriptors (zeros/ones left 0) and zeroed gaps between arrays
hipError_t wv_write_header(uint8_t* image, const wv_layout_in& in, hipStream_t s);
// status word: set when a symbol >= sigma is found
hipError_t wv_validate(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma,
                       uint8_t* image, uint64_t* counts /*nullable*/, hipStream_t s);
hipError_t wv_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s);
