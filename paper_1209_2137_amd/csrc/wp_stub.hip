// Temporary placeholders for entry points still being written.
#include "wp_host.hpp"
extern "C" int32_t bp_encode(const uint32_t *, uint64_t, int32_t, uint32_t *, uint64_t, uint64_t *, void *) { return WP_ERR_INVALID_ARG; }
extern "C" int32_t fastpfor_encode(const uint32_t *, uint64_t, int32_t, uint32_t *, uint64_t, uint64_t *, void *) { return WP_ERR_INVALID_ARG; }
extern "C" int32_t wp_batch_plan(const uint32_t *, uint32_t *, const wp_list *, uint64_t, const wp_tune *, void **, void *) { return WP_ERR_INVALID_ARG; }
extern "C" int32_t wp_batch_decode(void *, void *) { return WP_ERR_INVALID_ARG; }
extern "C" uint64_t wp_batch_items(const void *) { return 0; }
extern "C" int32_t wp_batch_free(void *) { return WP_ERR_INVALID_ARG; }
