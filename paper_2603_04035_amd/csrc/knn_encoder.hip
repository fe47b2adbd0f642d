// Learned seeding (encoder MLP, sorted projections) and the BF16 local join.
// Placeholder entry points until the kernels land.
#include "knn_common.hpp"

namespace knn {
knn_status encoder_seed(const knn_encoder*, const knn_matrix&, int, int, int, uint64_t, Workspace&,
                        int32_t**, float**, hipStream_t)
{
    return fail(KNN_ENOTSUP, "encoder seeding not built yet");
}
int encoder_dim(const knn_encoder*) { return -1; }
}  // namespace knn

using namespace knn;
extern "C" {
knn_status knn_encoder_create(int32_t, uint64_t, knn_encoder** enc)
{
    if (enc) *enc = nullptr;
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
void knn_encoder_destroy(knn_encoder*) {}
knn_status knn_encoder_set_weights(knn_encoder*, const float*, const float*, const float*, const float*)
{
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
knn_status knn_encoder_get_weights(const knn_encoder*, float*, float*, float*, float*)
{
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
knn_status knn_encoder_embed(const knn_encoder*, knn_matrix, int32_t, float*, void*)
{
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
knn_status knn_encoder_grads(knn_encoder*, knn_matrix, const int32_t*, int32_t, float, float*, float*, void*)
{
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
void knn_train_default_params(knn_train_params* t)
{
    if (!t) return;
    t->steps = 2000; t->batch = 4096; t->lr = 1e-3f; t->beta1 = 0.9f; t->beta2 = 0.999f;
    t->eps = 1e-8f; t->margin = 1.0f; t->seed = 0;
}
knn_status knn_encoder_train(knn_encoder*, knn_matrix, const int32_t*, int32_t, const knn_train_params*, float*, void*)
{
    return fail(KNN_ENOTSUP, "encoder not built yet");
}
knn_status knn_proj_seed(knn_matrix, const float*, int32_t, const float*, int32_t, int32_t, int32_t, int32_t*, float*, void*)
{
    return fail(KNN_ENOTSUP, "projection seeding not built yet");
}
}
