// Device-side entry points used by the C ABI (implemented in kernels.hip).
#pragma once

#include "hbc_internal.hpp"

namespace hbc {

void device_upload_plan(Plan& p);   // allocate and copy every table
void device_upload_tiles(Plan& p);  // tile table after a tuning change
void device_upload_csc(Plan& p);    // adjoint tables (built lazily)
void device_free_plan(Plan& p);
void device_apply(const Plan& p, void* field, void* stream, bool zero_only);
void device_update_b(Plan& p, int64_t first, int64_t last, void* stream);  // host.bval[first, last) to the device
void device_adjoint(const Plan& p, void* grad, void* stream);
void device_adjoint_noalloc(const Plan& p, void* grad, void* stream);  // counters in the static scratch
// demangled names of the kernels one apply (op HBC_OP_APPLY) or adjoint launches, in launch order
std::vector<std::string> device_kernel_names(const Plan& p, int op);
void device_stencil27(Plan& p, const void* x, void* y, void* stream, bool fused, void* xghost);
void* device_consumer_upload(const Plan& p, const ConsumerHost& C);  // the consumer's device tables
void device_consumer_free(void* h);
void device_consumer_apply(const Plan& p, const ConsumerHost& C, void* h, const void* x, void* y, bool fused,
                           void* stream);
void device_cs_weights(int64_t N, int64_t h, int32_t* base, double* w, void* stream);
double device_time_apply(const Plan& p, void* const* fields, int nfields, int reps, void* stream);
double device_plan_autotune(Plan& p, void* const* fields, int nfields, const char* cache_path, void* stream);
void* device_graph_create(const Plan& p, int op, void* const* fields, int nfields, int reps, void* stream);
void device_graph_launch(void* g, void* stream);
void device_graph_destroy(void* g);

struct Batch;
Batch* device_batch_create(Plan* const* plans, int n);
void device_batch_destroy(Batch* b);
void device_batch_bind(Batch* b, void* const* fields);
void device_batch_apply(Batch* b, void* stream);
void device_batch_capture(Batch* b, void* stream);
void device_batch_launch_graph(Batch* b, void* stream);
hbc_tune device_batch_get_tune(const Batch* b);
void device_batch_set_tune(Batch* b, const hbc_tune& t);
double device_batch_autotune(Batch* b, const char* cache_path, void* stream);
void device_batch_stats(const Batch* b, hbc_stats* out);

}  // namespace hbc
