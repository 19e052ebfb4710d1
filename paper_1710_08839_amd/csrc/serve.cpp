// placeholder, replaced by the serving scheduler
#include "host.h"
extern "C" {
qxd_status qxd_serve_start(qxd_ctx *, size_t, int) { qxd::set_error("serving not built"); return QXD_EINVAL; }
qxd_status qxd_serve_submit(qxd_ctx *, const qxd_request *, uint64_t *) { qxd::set_error("serving not built"); return QXD_EINVAL; }
qxd_status qxd_serve_poll(qxd_ctx *, uint64_t, qxd_result *) { qxd::set_error("serving not built"); return QXD_EINVAL; }
qxd_status qxd_serve_stop(qxd_ctx *) { return QXD_OK; }
}
