// wv_batch.hip -- batched wavelet-matrix builds over many sequences.
#include "wv_internal.h"

extern "C" {

int wt_batch_plan(int kind, const wt_seq_desc* seqs, uint32_t count, const wt_tuning* tune,
                  uint64_t* workspace_bytes)
{
    if (kind != WT_KIND_WM || (!seqs && count) || !workspace_bytes) return WT_EINVAL;
    uint64_t ws = 0;
    for (uint32_t i = 0; i < count; i++) {
        wt_plan_info info;
        int rc = wt_plan(WT_KIND_WM, seqs[i].n, seqs[i].sigma, seqs[i].sym_bytes, nullptr, tune, &info);
        if (rc) return rc;
        if (seqs[i].out_bytes < info.out_bytes) return WT_ENOSPC;
        ws = info.workspace_bytes > ws ? info.workspace_bytes : ws;
    }
    *workspace_bytes = ws;
    return WT_OK;
}

int wt_batch_build(int kind, const wt_seq_desc* seqs, uint32_t count, void* ws, size_t ws_bytes,
                   const wt_tuning* tune, void* stream)
{
    uint64_t need = 0;
    int rc = wt_batch_plan(kind, seqs, count, tune, &need);
    if (rc) return rc;
    if (ws_bytes < need) return WT_ENOSPC;
    for (uint32_t i = 0; i < count; i++) {
        rc = wm_build(seqs[i].S, seqs[i].n, seqs[i].sigma, seqs[i].sym_bytes, nullptr, tune, seqs[i].out,
                      seqs[i].out_bytes, ws, ws_bytes, stream);
        if (rc) return rc;
    }
    return WT_OK;
}

}  // extern "C"
