// engine.cpp -- placeholder until the engine lands.
#include "aesctr_internal.h"

extern "C" {
int aes_engine_create(const aes_engine_cfg_t *, aes_engine_t **) { return AES_EDEVICE; }
int aes_engine_destroy(aes_engine_t *) { return AES_EINVAL; }
int aes_submit(aes_engine_t *, const aes_ctr_desc_t *, uint64_t *) { return AES_EINVAL; }
int aes_poll(aes_engine_t *, uint64_t) { return AES_EINVAL; }
int aes_wait(aes_engine_t *, uint64_t, int64_t) { return AES_EINVAL; }
int aes_engine_stats(aes_engine_t *, aes_stats_t *) { return AES_EINVAL; }
int aes_engine_reset_stats(aes_engine_t *) { return AES_EINVAL; }
int aes_engine_completion_fd(aes_engine_t *) { return AES_EINVAL; }
}
