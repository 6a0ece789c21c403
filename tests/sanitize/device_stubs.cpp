// Device entry points for a host-only build of the library (the sanitizer
// test): every one refuses with HBC_EUNSUPPORTED, except freeing, which has
// nothing to free.  Host-only plans (HBC_PLAN_HOST_ONLY) never reach them.
#include "device.hpp"

namespace hbc {

namespace {
[[noreturn]] void no_device() { fail(HBC_EUNSUPPORTED, "host-only build: no device"); }
}  // namespace

void device_upload_plan(Plan&) { no_device(); }
void device_upload_tiles(Plan&) { no_device(); }
void device_upload_csc(Plan&) { no_device(); }
void device_free_plan(Plan&) {}
void device_apply(const Plan&, void*, void*, bool) { no_device(); }
void device_update_b(Plan&, int64_t, int64_t, void*) { no_device(); }
void device_adjoint(const Plan&, void*, void*) { no_device(); }
void device_adjoint_noalloc(const Plan&, void*, void*) { no_device(); }
std::vector<std::string> device_kernel_names(const Plan&, int) { no_device(); }
void device_stencil27(Plan&, const void*, void*, void*, bool, void*) { no_device(); }
void* device_consumer_upload(const Plan&, const ConsumerHost&) { no_device(); }
void device_consumer_free(void*) {}
void device_consumer_apply(const Plan&, const ConsumerHost&, void*, const void*, void*, bool, void*) { no_device(); }
void device_cs_weights(int64_t, int64_t, int32_t*, double*, void*) { no_device(); }
double device_time_apply(const Plan&, void* const*, int, int, void*) { no_device(); }
double device_plan_autotune(Plan&, void* const*, int, const char*, void*) { no_device(); }
void* device_graph_create(const Plan&, int, void* const*, int, int, void*) { no_device(); }
void device_graph_launch(void*, void*) { no_device(); }
void device_graph_destroy(void*) {}
Batch* device_batch_create(Plan* const*, int) { no_device(); }
void device_batch_destroy(Batch*) {}
void device_batch_bind(Batch*, void* const*) { no_device(); }
void device_batch_apply(Batch*, void*) { no_device(); }
void device_batch_capture(Batch*, void*) { no_device(); }
void device_batch_launch_graph(Batch*, void*) { no_device(); }
hbc_tune device_batch_get_tune(const Batch*) { no_device(); }
void device_batch_set_tune(Batch*, const hbc_tune&) { no_device(); }
double device_batch_autotune(Batch*, const char*, void*) { no_device(); }
void device_batch_stats(const Batch*, hbc_stats*) { no_device(); }

}  // namespace hbc
