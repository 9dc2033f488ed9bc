// Batched execution of many independent plans (declared in the C ABI).  Until the
// persistent batched launch exists, every entry point reports NFFT_ERR_UNSUPPORTED.
#include "../../include/nfft_mi355x.h"

extern "C" {

int nfft_batch_create(nfft_batch *out, int count, const nfft_plan *plans, const char *tune_cache)
{
    (void)out;
    (void)count;
    (void)plans;
    (void)tune_cache;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_workspace_bytes(nfft_batch b, size_t *bytes)
{
    (void)b;
    (void)bytes;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_set_workspace(nfft_batch b, void *ws, size_t bytes)
{
    (void)b;
    (void)ws;
    (void)bytes;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_autotune(nfft_batch b, hipStream_t s)
{
    (void)b;
    (void)s;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_trafo(nfft_batch b, const void *const *fhat, void *const *f, hipStream_t s)
{
    (void)b;
    (void)fhat;
    (void)f;
    (void)s;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_adjoint(nfft_batch b, const void *const *f, void *const *hhat, hipStream_t s)
{
    (void)b;
    (void)f;
    (void)hhat;
    (void)s;
    return NFFT_ERR_UNSUPPORTED;
}
int nfft_batch_destroy(nfft_batch b)
{
    (void)b;
    return NFFT_ERR_UNSUPPORTED;
}

}  // extern "C"
