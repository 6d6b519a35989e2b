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

// ---- tracing -----------------------------------------------------------------
// WT_TRACE=1 in the environment: plans are logged to stderr ("[wt] " lines)
bool wv_trace_on();
void wv_trace(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// ---- pinned host staging -------------------------------------------------------
// Pinned host buffers for copies a build issues between launches (the tables
// a shaped tree build uploads, the descriptors of a batch): a copy from
// pageable memory holds the host until it completes.  Buffers are pooled
// until the process ends.  A build never waits for its copies: it retires
// the buffer, which records an event on the stream and returns the buffer to
// the pool once that event has completed (checked when a buffer is next
// taken).  Under stream capture the buffer is kept for good instead, since
// the captured copies read it at every replay of the graph.
class PinnedBuf {
public:
    // `s`: the stream the copies will be queued on (no completed-copy check
    // while it is being captured)
    // At most CAP buffers wait for their copies: a caller that runs further
    // ahead of the device waits for the oldest of them instead of allocating
    // more pinned memory (an allocation costs far more than a build's copies).
    static constexpr size_t CAP = 8;
    PinnedBuf(size_t bytes, hipStream_t s)
    {
        if (!bytes) return;   // nothing to hold
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        const bool capturing = hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
        std::lock_guard<std::mutex> lk(mu());
        if (!capturing) {
            reclaim();
            if (!take(bytes) && pending().size() >= CAP) {
                // wait for the oldest retired buffer (the events complete in
                // stream order on one stream; any completed one is reclaimed)
                (void)hipEventSynchronize(pending().front().done);
                reclaim();
            }
        }
        if (p_ || take(bytes)) return;
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
    void idle() { idle_ = true; }   // no copy from or into it is pending any more
    // copies from or into the buffer are queued on s: it goes back to the
    // pool when s has passed them (or never, while s is being captured)
    void retire(hipStream_t s)
    {
        if (!p_ || idle_) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;   // kept
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;   // kept
        if (hipEventRecord(e, s) != hipSuccess) {
            (void)hipEventDestroy(e);
            return;   // kept
        }
        std::lock_guard<std::mutex> lk(mu());
        pending().push_back(Pending{p_, n_, e});
    }
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;

private:
    struct Pending {
        void* p;
        size_t n;
        hipEvent_t done;
    };
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
    static std::vector<Pending>& pending()
    {
        static std::vector<Pending> v;
        return v;
    }
    // (under the lock) a pooled buffer of at least `bytes`, the smallest
    bool take(size_t bytes)
    {
        auto& fr = pool();
        size_t best = fr.size();
        for (size_t i = 0; i < fr.size(); i++)
            if (fr[i].second >= bytes && (best == fr.size() || fr[i].second < fr[best].second)) best = i;
        if (best == fr.size()) return false;
        p_ = fr[best].first;
        n_ = fr[best].second;
        fr.erase(fr.begin() + (long)best);
        return true;
    }
    // (under the lock) retired buffers whose copies are done back to the pool
    static void reclaim()
    {
        auto& pd = pending();
        size_t k = 0;
        for (size_t i = 0; i < pd.size(); i++) {
            if (hipEventQuery(pd[i].done) == hipSuccess) {
                (void)hipEventDestroy(pd[i].done);
                pool().push_back({pd[i].p, pd[i].n});
            } else {
                pd[k++] = pd[i];
            }
        }
        pd.resize(k);
    }
    void* p_ = nullptr;
    size_t n_ = 0;
    bool idle_ = false;
};

// Copy `bytes` from a pinned host buffer (hipHostMalloc) to device memory with
// a kernel that reads the host memory directly, ordered on s like any launch
// (no copy engine between the kernels of a build, and a kernel node when s is
// captured).  Both pointers 16-byte aligned.
hipError_t wv_upload(void* dst, const void* pinned, uint64_t bytes, hipStream_t s);

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
// status word of the image header: bit 0 a symbol >= sigma, bit 1 symbol
// counts that differ from those a shape gave
constexpr uint32_t WV_STATUS_RANGE = 1u;
constexpr uint32_t WV_STATUS_COUNTS = 2u;
// sets WV_STATUS_COUNTS when got[x] != want[x] for some x < sigma (dev arrays)
hipError_t wv_check_counts(const uint64_t* got, const uint64_t* want, uint32_t sigma, uint8_t* image, hipStream_t s);
