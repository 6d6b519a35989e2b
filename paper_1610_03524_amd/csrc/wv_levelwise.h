// wv_levelwise.h -- arguments of the one-level-per-pass builder.
#pragma once

#include "wv_internal.h"

#define WV_KEY_SYMBOL      0u   // bit l from the top of the symbol
#define WV_KEY_CODE        1u   // digit l (D bits) of the symbol's codeword
#define WV_KEY_DIGIT_MULTI 2u   // D-bit digit l from the top of the symbol

// How a symbol maps to its bit / digit on one level.
struct wv_keyfn {
    uint32_t mode, shift, level, D;
    const uint32_t* codes;   // WV_KEY_CODE: codeword per symbol
    const uint32_t* lens;    // WV_KEY_CODE: codeword length per symbol
};

__device__ inline uint32_t wv_digit(const wv_keyfn& f, uint32_t key)
{
    if (f.mode == WV_KEY_CODE) {
        const uint32_t len = f.lens[key];   // digits
        return (f.codes[key] >> (f.D * (len - 1 - f.level))) & ((1u << f.D) - 1u);
    }
    return (key >> f.shift) & ((1u << f.D) - 1u);
}

// Tree nodes of every level (ids global, root = 0): start of the node on its
// level, and per child (d per node) its start on the next level and its id
// (WV_LEAF|symbol for a leaf, WV_NONE when absent).
struct wv_node_table {
    const uint32_t* start;
    const uint32_t* child_start;
    const uint32_t* child;
};

struct wv_lw_args {
    int kind;
    uint32_t arity_log2, key_bits, nlevels;
    const void* S;
    uint8_t* image;
    const wv_layout_out* lay;
    uint32_t *keys_a, *keys_b, *nodes_a, *nodes_b;
    wv_dir_scratch dir;
    wv_mdir_scratch mdir;
    uint64_t* zl;
    wv_node_table nt;
    const uint32_t* codes;
    const uint32_t* lens;
    bool profile;
    wv_keyfn keyfn(uint32_t l) const;
};

hipError_t wv_run_levelwise(const wv_lw_args& a, uint32_t sym_bytes, hipStream_t s);
