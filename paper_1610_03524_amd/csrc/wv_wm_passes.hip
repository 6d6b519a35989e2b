// wv_wm_passes.hip -- multi-level partition passes for the wavelet matrix.
#include "wv_wm_passes.h"

int wv_wm_make_plan(uint64_t, uint32_t, uint32_t, const wt_tuning*, wv_wm_plan& p)
{
    p.enabled = false;
    p.tau = 1;
    p.ws_bytes = 0;
    return WT_OK;
}

hipError_t wv_wm_run(const wv_wm_plan&, const void*, uint8_t*, const wv_layout_out&, uint8_t*,
                     const wv_dir_scratch&, hipStream_t)
{
    return hipErrorNotSupported;
}
