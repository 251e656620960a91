// fp32.hip -- placeholder of the batched FP32 form.
#include "fp32.h"

struct F32State {};

pic_status f32_init(pic_ctx* ctx) { pic_set_error(ctx, "FP32 form not available"); return PIC_EINVAL; }
void f32_destroy(pic_ctx*) {}
pic_status f32_load(pic_ctx*, int) { return PIC_EINVAL; }
pic_status f32_deposit_only(pic_ctx*, int) { return PIC_EINVAL; }
pic_status f32_step(pic_ctx*, int) { return PIC_EINVAL; }
pic_status f32_set_particles(pic_ctx*, int, long long, const double*, const double*, const double*,
                             const double*, const double*, const double*, const unsigned long long*) {
    return PIC_EINVAL;
}
pic_status f32_get_particles(pic_ctx*, int, double*, double*, double*, double*, double*, double*,
                             unsigned long long*, long long, long long*) {
    return PIC_EINVAL;
}
long long f32_live_count(pic_ctx*, int, const long long*) { return 0; }
pic_status f32_tuning(pic_ctx*, int*, int*, int*, int*, int*) { return PIC_EINVAL; }
