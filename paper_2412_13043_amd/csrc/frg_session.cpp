// Serving loop (continuous batching of flow right-hand-side requests).
#include "frg_runtime.hpp"

using namespace frg;

extern "C" {

frg_status frg_session_open(frg_context *, const frg_session_config *, frg_session **) {
    set_error("sessions are not built yet");
    return FRG_E_UNSUPPORTED;
}
frg_status frg_session_register_table(frg_session *, const double *, int, double, double, int *) {
    return FRG_E_UNSUPPORTED;
}
frg_status frg_session_submit(frg_session *, const frg_integral_desc *, const frg_batch *, int,
                              uint64_t *) {
    return FRG_E_UNSUPPORTED;
}
frg_status frg_session_poll(frg_session *, uint64_t, int *) { return FRG_E_UNSUPPORTED; }
frg_status frg_session_wait(frg_session *, uint64_t, int) { return FRG_E_UNSUPPORTED; }
frg_status frg_session_cancel(frg_session *, uint64_t) { return FRG_E_UNSUPPORTED; }
frg_status frg_session_stats(frg_session *, frg_stats *) { return FRG_E_UNSUPPORTED; }
frg_status frg_session_close(frg_session *) { return FRG_E_UNSUPPORTED; }

}  // extern "C"
