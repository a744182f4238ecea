// C ABI of the learned-proposal network: validation and workspace layout.
#include "labs_internal.h"

#include <climits>
#include <cmath>

using namespace labsdev;

namespace {

hipStream_t S(void* s) { return (hipStream_t)s; }

labs_status check_layout(const labs_mlp_layout* y) {
    if (!y) return invalid("layout must not be NULL");
    labs_mlp_layout ref;
    if (!mlp_layout(y->L, y->hidden, &ref)) return invalid("layout: unsupported L=%d hidden=%d", y->L, y->hidden);
    if (ref.n_params != y->n_params || ref.off_W3 != y->off_W3 || ref.ld_in != y->ld_in ||
        ref.ld_out != y->ld_out || ref.d_in != y->d_in || ref.d_out != y->d_out)
        return invalid("layout was not produced by labs_mlp_layout_of");
    return LABS_OK;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

labs_status check_rows(int64_t n) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return invalid("n must be in [0, 2^30)");
    return LABS_OK;
}

labs_status check_adam(int32_t t, double lr, double b1, double b2, double eps) {
    if (t < 1) return invalid("Adam step t counts from 1");
    if (!(b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1)) return invalid("betas must lie in [0, 1)");
    if (!(lr >= 0 && std::isfinite(lr)) || !(eps > 0 && std::isfinite(eps)))
        return invalid("lr must be finite and >= 0, eps finite and > 0");
    return LABS_OK;
}

labs_status check_learned(const labs_step1_cfg* cfg, const labs_proposer* pr) {
    if (!cfg || !pr) return invalid("cfg and prop must not be NULL");
    if (labs_status s = validate_step1_cfg(*cfg)) return s;
    if (cfg->flags != 0) return invalid("flags must be 0 for the learned walk");
    if (!learned_walk_supported(cfg->L)) return invalid("learned walk needs L <= 639");
    if (pr->mode != LABS_PROPOSE_MLP && pr->mode != LABS_PROPOSE_RANDOM) return invalid("unknown proposer mode");
    if (pr->top_m < 1 || pr->top_m > 64) return invalid("top_m must be in [1, 64]");
    if (pr->fallback_every < 1) return invalid("fallback_every must be >= 1");
    if (pr->log_every < 0) return invalid("log_every must be >= 0");
    if (pr->reserved != 0) return invalid("reserved must be 0");
    if (pr->mode == LABS_PROPOSE_MLP) {
        labs_mlp_layout y;
        if (!mlp_layout(cfg->L, pr->hidden, &y)) return invalid("unsupported network width %d", pr->hidden);
        if (!pr->params || !pr->params_bf16) return invalid("network parameters must not be NULL");
        if (!aligned16(pr->params_bf16)) return invalid("params_bf16 must be 16-byte aligned");
    }
    return LABS_OK;
}

labs_step1_cfg with_default_steps(const labs_step1_cfg& c) {
    labs_step1_cfg r = c;
    if (r.steps == 0) r.steps = 4 * (r.L + 1);   // T_i = 4(L+1), as labs_walk_step1
    return r;
}

}  // namespace

extern "C" {

labs_status labs_learned_walk_workspace(const labs_step1_cfg* cfg, const labs_proposer* prop, size_t* bytes) {
    clear_error();
    if (labs_status s = check_learned(cfg, prop)) return s;
    if (!bytes) return invalid("bytes must not be NULL");
    *bytes = learned_walk_ws(with_default_steps(*cfg), *prop);
    return LABS_OK;
}

labs_status labs_learned_walk(const labs_step1_cfg* cfg, const labs_proposer* prop, const labs_learned_out* out,
                              void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (labs_status s = check_learned(cfg, prop)) return s;
    if (!out || !out->flip_evals) return invalid("out and out->flip_evals must not be NULL");
    if (prop->log_every > 0 && cfg->steps / prop->log_every > 0 &&
        (!out->log_seqs || !out->log_mask || !out->log_label))
        return invalid("log_every > 0 needs log_seqs, log_mask and log_label");
    const labs_step1_cfg c = with_default_steps(*cfg);
    if (!ws || ws_bytes < learned_walk_ws(c, *prop)) return invalid("workspace too small");
    return learned_walk(c, *prop, *out, ws, ws_bytes, S(stream));
}

labs_status labs_mlp_layout_of(int32_t L, int32_t hidden, labs_mlp_layout* out) {
    clear_error();
    if (!out) return invalid("out must not be NULL");
    if (!mlp_layout(L, hidden, out))
        return invalid("MLP needs odd L in [5, 1023] and hidden a multiple of 64 in [64, 1024] (L=%d hidden=%d)",
                       L, hidden);
    return LABS_OK;
}

labs_status labs_mlp_features(int32_t L, int64_t n, const uint32_t* seqs, uint16_t* X, void* stream) {
    clear_error();
    labs_mlp_layout y;
    if (!mlp_layout(L, 64, &y)) return invalid("features need odd L in [5, 1023], got %d", L);
    if (labs_status s = check_rows(n)) return s;
    if (n > 0 && (!seqs || !X)) return invalid("seqs and X must not be NULL");
    return launch_features(L, n, seqs, X, y.ld_in, S(stream));
}

labs_status labs_mlp_forward_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (!bytes) return invalid("bytes must not be NULL");
    *bytes = mlp_forward_ws(*lay, n);
    return LABS_OK;
}

labs_status labs_mlp_forward(const labs_mlp_layout* lay, const float* params, const uint16_t* params_bf16,
                             int64_t n, const uint16_t* X, float* logits, void* ws, size_t ws_bytes,
                             void* stream) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (n == 0) return LABS_OK;
    if (!params || !params_bf16 || !X || !logits || !ws) return invalid("pointers must not be NULL");
    if (!aligned16(params_bf16) || !aligned16(X)) return invalid("params_bf16 and X must be 16-byte aligned");
    if (ws_bytes < mlp_forward_ws(*lay, n)) return invalid("workspace too small");
    return mlp_forward(*lay, params, params_bf16, n, X, logits, ws, ws_bytes, S(stream));
}

labs_status labs_mlp_grads_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (!bytes) return invalid("bytes must not be NULL");
    *bytes = mlp_grads_ws(*lay, n);
    return LABS_OK;
}

labs_status labs_mlp_grads(const labs_mlp_layout* lay, const float* params, const uint16_t* params_bf16,
                           int64_t n, const uint16_t* X, const uint32_t* mask, const int32_t* labels,
                           float* grads, float* loss, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (!params || !params_bf16 || !grads || !loss || !ws) return invalid("pointers must not be NULL");
    if (n > 0 && (!X || !mask || !labels)) return invalid("X, mask and labels must not be NULL");
    if (!aligned16(params_bf16) || (X && !aligned16(X))) return invalid("params_bf16 and X must be 16-byte aligned");
    if (ws_bytes < mlp_grads_ws(*lay, n)) return invalid("workspace too small");
    return mlp_grads(*lay, params, params_bf16, n, X, mask, labels, grads, loss, ws, ws_bytes, S(stream));
}

labs_status labs_mlp_adam(const labs_mlp_layout* lay, float* params, uint16_t* params_bf16, const float* grads,
                          float* m, float* v, int32_t t, double lr, double beta1, double beta2, double eps,
                          void* stream) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_adam(t, lr, beta1, beta2, eps)) return s;
    if (!params || !params_bf16 || !grads || !m || !v) return invalid("pointers must not be NULL");
    return mlp_adam(*lay, params, params_bf16, grads, m, v, t, lr, beta1, beta2, eps, S(stream));
}

labs_status labs_mlp_cast(const labs_mlp_layout* lay, const float* params, uint16_t* params_bf16, void* stream) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (!params || !params_bf16) return invalid("pointers must not be NULL");
    return mlp_cast(*lay, params, params_bf16, S(stream));
}

labs_status labs_mlp_train_workspace(const labs_mlp_layout* lay, int64_t n, size_t* bytes) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (!bytes) return invalid("bytes must not be NULL");
    *bytes = align_up((size_t)n * lay->ld_in * 2, 256) + mlp_grads_ws(*lay, n);
    return LABS_OK;
}

labs_status labs_mlp_train_step(const labs_mlp_layout* lay, float* params, uint16_t* params_bf16, float* grads,
                                float* m, float* v, int32_t t, double lr, double beta1, double beta2, double eps,
                                int64_t n, const uint32_t* seqs, const uint32_t* mask, const int32_t* labels,
                                float* loss, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (labs_status s = check_layout(lay)) return s;
    if (labs_status s = check_rows(n)) return s;
    if (labs_status s = check_adam(t, lr, beta1, beta2, eps)) return s;
    if (!params || !params_bf16 || !grads || !m || !v || !loss || !ws) return invalid("pointers must not be NULL");
    if (n > 0 && (!seqs || !mask || !labels)) return invalid("seqs, mask and labels must not be NULL");
    if (!aligned16(params_bf16)) return invalid("params_bf16 must be 16-byte aligned");
    const size_t xb = align_up((size_t)n * lay->ld_in * 2, 256);
    if (ws_bytes < xb + mlp_grads_ws(*lay, n)) return invalid("workspace too small");
    if (!aligned16(ws)) return invalid("workspace must be 16-byte aligned");
    uint16_t* X = (uint16_t*)ws;
    labs_status s = launch_features(lay->L, n, seqs, X, lay->ld_in, S(stream));
    if (s) return s;
    s = mlp_grads(*lay, params, params_bf16, n, X, mask, labels, grads, loss, (char*)ws + xb, ws_bytes - xb,
                  S(stream));
    if (s) return s;
    return mlp_adam(*lay, params, params_bf16, grads, m, v, t, lr, beta1, beta2, eps, S(stream));
}

}  // extern "C"
