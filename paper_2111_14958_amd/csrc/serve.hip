// Serving engine (placeholder).
#include "cg_host.h"
extern "C" {
size_t wd_serve_footprint(const wd_request *) { return 0; }
int wd_serve_create(const wd_serve_config *, wd_server **) { return WD_EINVAL; }
int wd_serve_submit(wd_server *, const wd_request *, uint64_t *) { return WD_EINVAL; }
int wd_serve_poll(wd_server *, uint64_t, wd_cg_report *, int32_t *) { return WD_EINVAL; }
int wd_serve_stats_get(wd_server *, wd_serve_stats *) { return WD_EINVAL; }
int wd_serve_destroy(wd_server *) { return WD_EINVAL; }
}
