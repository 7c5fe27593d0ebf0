// The state store (every recurrence state T_0 R .. T_p R kept) as seen from
// translation units that do not launch recurrence steps themselves.
#pragma once

#include "common.hpp"

namespace asc {

// Panel layout: slice sl holds columns [sl*rs, sl*rs + rs) of every state;
// state j of slice sl is an n x rs row-major panel at byte offset
// (sl*(p+1) + j) * panel_bytes of the store.
struct StoreLayout {
    int rs;
    int nslices;
    size_t panel_bytes;
};
StoreLayout store_layout(const asc_graph *g, int64_t r, asc_dtype sig);
size_t store_ws_bytes(int64_t n, int64_t r, asc_dtype sig);
// Runs the recurrence of every slice of R into the store (no Y, no moments).
// The store holds asc_ckpt_bytes(g, r, sig, p, 1) bytes.
asc_status run_store(const asc_graph *g, const double *lmax, int p, const void *R, asc_dtype sig, int64_t r,
                     int64_t ldr, void *states, void *ws, hipStream_t s);

}  // namespace asc
