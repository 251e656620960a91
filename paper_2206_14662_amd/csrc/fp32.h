// fp32.h -- the batched FP32 form: tile-sorted SoA FP32 particles, one fused
// persistent particle kernel per step with LDS charge accumulation, periodic
// tile sort, captured step graphs.
#pragma once

#include <string>

#include "pic_internal.h"

struct F32State;

// accessors of the context (api.hip)
void* pic_dev_alloc(pic_ctx* ctx, size_t bytes);
void pic_dev_free(pic_ctx* ctx, void* p);
hipStream_t pic_stream(pic_ctx* ctx);
// instance k exists (PIC_OK) or the error recorded on ctx
pic_status pic_check_instance(pic_ctx* ctx, int k);
// record an error message on ctx and return st
pic_status pic_fail(pic_ctx* ctx, pic_status st, const std::string& msg);
int pic_device(pic_ctx* ctx);
long long pic_inst_nodes(pic_ctx* ctx, int k);
const double* pic_inst_volume(pic_ctx* ctx, int k);   // device node volumes
// launch the moment kernels of instance k into acc (kMoments channel-major
// node arrays, zeroed by the caller) on the context's stream; no allocation
pic_status pic_moments_accumulate(pic_ctx* ctx, int k, double* acc);
int pic_n_inst(pic_ctx* ctx);
pic::DevInst& pic_inst_dev(pic_ctx* ctx, int k);
const pic_instance_cfg& pic_inst_cfg(pic_ctx* ctx, int k);
long long* pic_counters(pic_ctx* ctx);
long long* pic_inst_Q(pic_ctx* ctx, int k);
float4* pic_inst_EB(pic_ctx* ctx, int k);
pic::DevInst* pic_dev_table(pic_ctx* ctx);
// copies the host instance table (after p_off/p_cap/tile changes) to the device
pic_status pic_upload_inst(pic_ctx* ctx);
long long* pic_inst_Qw(pic_ctx* ctx, int k);
long long* pic_inst_Qx(pic_ctx* ctx, int k);
pic_status f32_rates_changed(pic_ctx* ctx);
long long& pic_inst_cap(pic_ctx* ctx, int k);
const pic_run_cfg& pic_run(pic_ctx* ctx);
void pic_set_error(pic_ctx* ctx, const std::string& m);
bool pic_timing_on(pic_ctx* ctx);
hipEvent_t pic_timing_begin(pic_ctx* ctx, hipEvent_t* stop);
void pic_set_f32(pic_ctx* ctx, F32State* s);
F32State* pic_get_f32(pic_ctx* ctx);
pic_status pic_solve_all(pic_ctx* ctx);
// the FP32 step plan (control words) the end-of-step kernel refreshes
void pic_set_prep_ctl(pic_ctx* ctx, long long* ctl);
// FP64 field solve, nodal E, diagnostics sample and step commit on stream s
pic_status pic_field_stage(pic_ctx* ctx, hipStream_t s);
pic::FieldDev* pic_field_table(pic_ctx* ctx);

// the FP32 form (fp32.hip)
pic_status f32_init(pic_ctx* ctx);
void f32_destroy(pic_ctx* ctx);
pic_status f32_load(pic_ctx* ctx, int k);
pic_status f32_deposit_only(pic_ctx* ctx, int k);
pic_status f32_step(pic_ctx* ctx, int n_steps);
pic_status f32_sort_now(pic_ctx* ctx);
pic_status f32_set_particles(pic_ctx* ctx, int k, long long n, const double* r, const double* z,
                             const double* vr, const double* vt, const double* vz, const double* w,
                             const unsigned long long* key);
pic_status f32_get_particles(pic_ctx* ctx, int k, double* r, double* z, double* vr, double* vt,
                             double* vz, double* w, unsigned long long* key, long long cap,
                             long long* n_out);
pic_status f32_check(pic_ctx* ctx);
long long f32_live_count(pic_ctx* ctx, int k, const long long* cnt);
pic_status f32_tuning(pic_ctx* ctx, int* tile_r, int* tile_z, int* halo, int* sort_interval, int* chunk,
                      int* lanes, int* use_graph);
pic_status f32_retune(pic_ctx* ctx, int tile_r, int tile_z, int halo, int sort_interval);
pic_status f32_reserve(pic_ctx* ctx, int k, long long slots);
pic_status f32_autotune(pic_ctx* ctx, int trial_steps, const char* cache, int out[4], double* ms_out,
                        int* trials_out);
long long f32_grow_events(pic_ctx* ctx);
// fluid-moment node sums of instance k into acc (kMoments x nodes, zeroed)
pic_status f32_moments(pic_ctx* ctx, int k, double* acc);
