#include "sf_internal.hpp"
namespace sf {
}
extern "C" {
int sf_batch_create(sf_context *, const sf_job *, int32_t, sf_batch **) { return SF_ERR_UNSUPPORTED; }
int sf_batch_launch(sf_batch *, void *) { return SF_ERR_UNSUPPORTED; }
int sf_batch_destroy(sf_batch *) { return SF_ERR_UNSUPPORTED; }
int sf_batch_info(const sf_batch *, int64_t *, int32_t *) { return SF_ERR_UNSUPPORTED; }
int sf_autotune(sf_context *, const sf_op *, int64_t, const char *) { return SF_ERR_UNSUPPORTED; }
int sf_tuned_variant(sf_context *, const sf_op *, int32_t *) { return SF_ERR_UNSUPPORTED; }
int sf_load_tuning(sf_context *, const char *) { return SF_ERR_UNSUPPORTED; }
}
