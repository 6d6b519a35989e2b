// wv_wm_passes.h -- multi-level partition passes for the wavelet matrix.
#pragma once

#include "wv_internal.h"

struct wv_wm_plan {
    bool enabled;          // false: the one-level-per-pass builder is used
    uint32_t tau;          // key bits (levels) handled per pass
    uint32_t L, sym_bytes, K, C, sigma;
    uint64_t n;
    // workspace offsets
    uint64_t off_H, off_tot, off_G0, off_pay[2], off_dir;
    wv_span_dir dir;
    uint64_t ws_bytes;     // workspace the passes need
    bool profile;          // bracket the launches with timing events
    // Place every run of every level in key order: the levels of a balanced
    // tree built directly when one pass covers all its key bits (the domain
    // decomposition of Sec. 4.2: every chunk's runs go to their node at the
    // node's start plus the node's symbols in earlier chunks)
    bool tree_order;
};

// Decide how the multi-level passes build this matrix.
int wv_wm_make_plan(uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_tuning* tune, wv_wm_plan& p);

// The level bits only: level l's words go to level_words[l] (host array of
// device pointers, ceil(n/64) words each); a symbol >= sigma sets *status.
hipError_t wv_wm_levels(const wv_wm_plan& p, const void* S, uint64_t* const* level_words, uint32_t* status,
                        uint8_t* ws, hipStream_t s);

// Build every level, directory and select sample of the matrix into `image`.
hipError_t wv_wm_run(const wv_wm_plan& p, const void* S, uint8_t* image, const wv_layout_out& lay,
                     uint8_t* ws, const wv_dir_scratch& dir, hipStream_t s);
