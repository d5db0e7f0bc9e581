// Batched d = 1 transforms (placeholder until the persistent batched kernels land).
#include "blnfft_internal.h"

struct bl_batch_s {
    int count;
};

extern "C" {

bl_status bl_batch_create(bl_batch* out, int count, const int64_t* M, const int64_t* L,
                          const int* m, const int64_t* N, bl_precision prec, void* stream) {
    (void)count; (void)M; (void)L; (void)m; (void)N; (void)prec; (void)stream;
    if (out) *out = nullptr;
    bl::set_error("batched transforms are not available in this build");
    return BL_EUNSUPPORTED;
}

bl_status bl_batch_set_nodes(bl_batch batch, const void* x_dev) {
    (void)batch; (void)x_dev;
    bl::set_error("batched transforms are not available in this build");
    return BL_EUNSUPPORTED;
}

bl_status bl_batch_forward(bl_batch batch, const void* fhat_dev, void* f_dev) {
    (void)batch; (void)fhat_dev; (void)f_dev;
    bl::set_error("batched transforms are not available in this build");
    return BL_EUNSUPPORTED;
}

bl_status bl_batch_destroy(bl_batch batch) {
    (void)batch;
    return BL_OK;
}

}  // extern "C"
