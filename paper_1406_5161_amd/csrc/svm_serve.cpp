// svm_serve.cpp -- batched training and the serving loop (continuous batching).
#include "svm_internal.h"

extern "C" {

int svm_train_batch(int32_t, const svm_problem_t*, const svm_params_t*, double* const*, double* const*,
                    svm_result_t*, void*) {
    return SVM_EUNSUPPORTED;
}
int svm_server_create(size_t, int32_t, void**) { return SVM_EUNSUPPORTED; }
int svm_server_submit(void*, const svm_problem_t*, const svm_params_t*, double*, int64_t*) { return SVM_EUNSUPPORTED; }
int svm_server_poll(void*, int64_t, svm_result_t*) { return SVM_EUNSUPPORTED; }
int svm_server_drain(void*) { return SVM_EUNSUPPORTED; }
int svm_server_stats(void*, int64_t*, int64_t*, int64_t*, int64_t*) { return SVM_EUNSUPPORTED; }
int svm_server_destroy(void*) { return SVM_EUNSUPPORTED; }

}  // extern "C"
