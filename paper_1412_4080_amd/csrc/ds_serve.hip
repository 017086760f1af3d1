// Serving entry points (continuous batching) - filled in by the serving engine.
#include <hip/hip_runtime.h>

#include "ds_engine.h"

using namespace ds;

extern "C" {
ds_status ds_server_create(const ds_server_config*, void**) { set_error("serving not built"); return DS_EINVAL; }
ds_status ds_server_add_dict(void*, const ds_problem*, ds_dtype, int32_t*) { set_error("serving not built"); return DS_EINVAL; }
ds_status ds_submit(void*, int32_t, const void*, double, const ds_params*, uint64_t*) { set_error("serving not built"); return DS_EINVAL; }
ds_status lasso_submit(void*, int32_t, const void*, double, const ds_params*, uint64_t*) { set_error("serving not built"); return DS_EINVAL; }
ds_status lasso_poll(void*, uint64_t, void*, ds_info*) { set_error("serving not built"); return DS_EINVAL; }
ds_status ds_server_destroy(void*) { set_error("serving not built"); return DS_EINVAL; }
}
