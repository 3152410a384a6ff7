// C ABI entry points (see include/sdirt.h).  Each validates and resolves
// its arguments on the host, then enqueues the kernels on the caller's
// stream without synchronising.
#include <hip/hip_runtime.h>

#include <cmath>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/sdirt.h"
#include "host_optics.hpp"
#include "pack.hpp"

namespace sdirt {
int trace_dp_psf_impl(const sdirt_lens*, const sdirt_sensor*, const sdirt_psf_query*,
                      void*, double*, hipStream_t, int, const int*);
int trace_rays_impl(const sdirt_lens*, double, int, int, const double*, const double*,
                    double*, int*, hipStream_t);
int trace_backward_impl(const sdirt_lens*, const sdirt_sensor*, const sdirt_psf_query*,
                        const float*, double*, hipStream_t);
int render_impl(const sdirt_render_desc*, const float*, const void*, const float*,
                float*, hipStream_t);
int render_backward_impl(const sdirt_render_desc*, const void*, const float*,
                         const float*, float*, hipStream_t);
int render_psf_backward_impl(const sdirt_render_desc*, const float*, const float*, const float*,
                             void*, hipStream_t);
int mlp_n_params(const sdirt_mlp_desc*, long long*);
int mlp_workspace_size(const sdirt_mlp_desc*, int, size_t*);
int mlp_forward(const sdirt_mlp_desc*, const float*, long long, const float*, void*, int,
                void*, int, hipStream_t);
int mlp_render(const sdirt_mlp_desc*, const float*, const sdirt_mlp_render_desc*, const float*,
               const float*, float*, void*, int, hipStream_t);
int mlp_forward_noalloc(const sdirt_mlp_desc*, const float*, long long, const float*, void*, int,
                        hipStream_t);
int mlp_backward(const sdirt_mlp_desc*, const float*, int, const float*, const float*,
                 float*, float*, void*, hipStream_t);
int mlp_vjp(const sdirt_mlp_desc*, const float*, long long, const float*, const float*,
            float*, float*, void*, int, hipStream_t);
int mlp_adam(const sdirt_mlp_desc*, float*, float*, float*, const float*, int, float,
             hipStream_t);
int mlp_train(const sdirt_mlp_desc*, float*, float*, float*, int, int, float, float, int, int,
              long long, const float*, const float*, uint32_t, float*, void*, hipStream_t);
int mlp_train_step(const sdirt_mlp_desc*, float*, float*, float*, int, float, int, const float*,
                   const float*, float*, void*, hipStream_t);
int calib_fma64(long long, int, double*, hipStream_t);
int psf_hybrid(const sdirt_mlp_desc*, const float*, const sdirt_lens*, const sdirt_sensor*,
               const sdirt_psf_query*, int, const double*, const double*, double, float*, int*,
               void*, int, hipStream_t);
}  // namespace sdirt

using namespace sdirt;

namespace {
// A roctx range named after the entry point around each call that launches
// device work, so that profiler timelines (rocprofv3 --marker-trace) group
// the kernels by the C-ABI call that issued them.
struct Range {
    explicit Range(const char* name) { roctxRangePush(name); }
    ~Range() { roctxRangePop(); }
};
}  // namespace

extern "C" {

int sdirt_version(void) { return 1; }

const char* sdirt_status_string(int status) {
    switch (status) {
        case SDIRT_OK: return "ok";
        case SDIRT_EINVAL: return "invalid argument";
        case SDIRT_EUNSUPPORTED: return "unsupported mode, dtype or size";
        case SDIRT_ELAUNCH: return "HIP launch or runtime failure";
        case SDIRT_ENODEVICE: return "no HIP device";
        case SDIRT_ESCRATCH: return "needs more memory than the library's static scratch array";
        default: return "unknown status";
    }
}

int sdirt_resolve_lens(const sdirt_lens* lens, sdirt_lens_info* out) {
    if (!out) return SDIRT_EINVAL;
    Resolved R;
    const int rc = resolve_lens(lens, &R);
    if (rc) return rc;
    out->efl = R.efl;
    out->bfd = R.bfd;
    out->sensor_distance = R.sensor_distance;
    out->stop_radius = R.stop_radius;
    out->z_ep = R.z_ep_ref;
    out->rho_ep = R.rho_ep_ref;
    out->m_num = R.m_num;
    out->sensor_z = R.sensor_z;
    return SDIRT_OK;
}

int sdirt_pupil(const sdirt_lens* lens, double wavelength, double* z_ep, double* rho_ep) {
    if (!z_ep || !rho_ep || !std::isfinite(wavelength) || !(wavelength > 0)) return SDIRT_EINVAL;
    Resolved R;
    const int rc = resolve_lens(lens, &R);
    if (rc) return rc;
    for (int m = 0; m <= R.S; ++m)
        if (!(R.index(m, wavelength) > 0)) return SDIRT_EINVAL;
    R.pupil(wavelength, z_ep, rho_ep);
    return SDIRT_OK;
}

int sdirt_n_params(const sdirt_lens* lens) {
    if (!lens || lens->n_surfaces < 1 || lens->n_surfaces > SDIRT_MAX_SURFACES) return SDIRT_EINVAL;
    return 8 * lens->n_surfaces + 1;
}

int sdirt_trace_rays(const sdirt_lens* lens, double wavelength, int math, int n,
                     const double* o, const double* d, double* hits_out,
                     int* status_out, void* stream) {
    Range r("sdirt_trace_rays");
    return trace_rays_impl(lens, wavelength, math, n, o, d, hits_out, status_out,
                           (hipStream_t)stream);
}

int sdirt_trace_dp_psf(const sdirt_lens* lens, const sdirt_sensor* sensor,
                       const sdirt_psf_query* query, void* psf_out,
                       double* stats_out, void* stream) {
    Range r("sdirt_trace_dp_psf");
    return trace_dp_psf_impl(lens, sensor, query, psf_out, stats_out,
                             (hipStream_t)stream, 0, nullptr);
}

int sdirt_trace_dp_psf_chunks(const sdirt_lens* lens, const sdirt_sensor* sensor,
                              const sdirt_psf_query* query, void* psf_out,
                              double* stats_out, int chunks, void* stream) {
    Range r("sdirt_trace_dp_psf_chunks");
    if (chunks < 1) return SDIRT_EINVAL;
    return trace_dp_psf_impl(lens, sensor, query, psf_out, stats_out,
                             (hipStream_t)stream, chunks, nullptr);
}

int sdirt_trace_dp_psf_backward(const sdirt_lens* lens, const sdirt_sensor* sensor,
                                const sdirt_psf_query* query, const float* grad_psf,
                                double* grad_params_out, void* stream) {
    Range r("sdirt_trace_dp_psf_backward");
    return trace_backward_impl(lens, sensor, query, grad_psf, grad_params_out,
                               (hipStream_t)stream);
}

int sdirt_render_dp(const sdirt_render_desc* desc, const float* img, const void* psf,
                    const float* depth, float* out, void* stream) {
    Range r("sdirt_render_dp");
    return render_impl(desc, img, psf, depth, out, (hipStream_t)stream);
}

int sdirt_render_dp_backward(const sdirt_render_desc* desc, const void* psf,
                             const float* depth, const float* grad_out,
                             float* grad_img, void* stream) {
    Range r("sdirt_render_dp_backward");
    return render_backward_impl(desc, psf, depth, grad_out, grad_img, (hipStream_t)stream);
}

int sdirt_render_dp_psf_backward(const sdirt_render_desc* desc, const float* img,
                                 const float* depth, const float* grad_out,
                                 void* grad_psf, void* stream) {
    Range r("sdirt_render_dp_psf_backward");
    return render_psf_backward_impl(desc, img, depth, grad_out, grad_psf, (hipStream_t)stream);
}

int sdirt_mlp_n_params(const sdirt_mlp_desc* desc, long long* n_params) {
    if (!n_params) return SDIRT_EINVAL;
    return mlp_n_params(desc, n_params);
}

int sdirt_mlp_workspace_size(const sdirt_mlp_desc* desc, int batch, size_t* bytes) {
    if (!bytes) return SDIRT_EINVAL;
    return mlp_workspace_size(desc, batch, bytes);
}

int sdirt_mlp_forward(const sdirt_mlp_desc* desc, const float* params, long long n_rows,
                      const float* x, void* out, int out_dtype, void* workspace,
                      int ws_batch, void* stream) {
    Range r("sdirt_mlp_forward");
    return mlp_forward(desc, params, n_rows, x, out, out_dtype, workspace, ws_batch,
                       (hipStream_t)stream);
}

int sdirt_mlp_forward_noalloc(const sdirt_mlp_desc* desc, const float* params,
                              long long n_rows, const float* x, void* out, int out_dtype,
                              void* stream) {
    Range r("sdirt_mlp_forward_noalloc");
    return mlp_forward_noalloc(desc, params, n_rows, x, out, out_dtype, (hipStream_t)stream);
}

int sdirt_mlp_render(const sdirt_mlp_desc* desc, const float* params,
                     const sdirt_mlp_render_desc* render, const float* img,
                     const float* depth, float* out, void* workspace, int ws_batch,
                     void* stream) {
    Range r("sdirt_mlp_render");
    return mlp_render(desc, params, render, img, depth, out, workspace, ws_batch,
                      (hipStream_t)stream);
}

int sdirt_mlp_backward(const sdirt_mlp_desc* desc, const float* params, int batch,
                       const float* x, const float* target, float* grads_out,
                       float* loss_out, void* workspace, void* stream) {
    Range r("sdirt_mlp_backward");
    return mlp_backward(desc, params, batch, x, target, grads_out, loss_out, workspace,
                        (hipStream_t)stream);
}

int sdirt_mlp_vjp(const sdirt_mlp_desc* desc, const float* params, long long n_rows,
                  const float* x, const float* grad_psf, float* grads_out, float* value_out,
                  void* workspace, int ws_batch, void* stream) {
    Range r("sdirt_mlp_vjp");
    return mlp_vjp(desc, params, n_rows, x, grad_psf, grads_out, value_out, workspace,
                   ws_batch, (hipStream_t)stream);
}

int sdirt_mlp_adam(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                   const float* grads, int step, float lr, void* stream) {
    Range r("sdirt_mlp_adam");
    return mlp_adam(desc, params, m, v, grads, step, lr, (hipStream_t)stream);
}

int sdirt_mlp_train_step(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                         int step, float lr, int batch, const float* x, const float* target,
                         float* loss_out, void* workspace, void* stream) {
    Range r("sdirt_mlp_train_step");
    return mlp_train_step(desc, params, m, v, step, lr, batch, x, target, loss_out, workspace,
                          (hipStream_t)stream);
}

int sdirt_mlp_train(const sdirt_mlp_desc* desc, float* params, float* m, float* v,
                    int step0, int n_steps, float lr0, float lr_min, int total_steps,
                    int batch, long long n_samples, const float* x_all,
                    const float* t_all, uint32_t seed, float* loss_trace,
                    void* workspace, void* stream) {
    Range r("sdirt_mlp_train");
    return mlp_train(desc, params, m, v, step0, n_steps, lr0, lr_min, total_steps, batch,
                     n_samples, x_all, t_all, seed, loss_trace, workspace,
                     (hipStream_t)stream);
}

int sdirt_psf_hybrid(const sdirt_mlp_desc* desc, const float* params, const sdirt_lens* lens,
                     const sdirt_sensor* sensor, const sdirt_psf_query* query, int n_bands,
                     const double* band_edges, const double* band_error, double max_error,
                     float* psf_out, int* source_out, void* workspace, int ws_batch,
                     void* stream) {
    Range r("sdirt_psf_hybrid");
    return psf_hybrid(desc, params, lens, sensor, query, n_bands, band_edges, band_error,
                      max_error, psf_out, source_out, workspace, ws_batch, (hipStream_t)stream);
}

int sdirt_calib_fma64(long long n_threads, int iters, double* out, void* stream) {
    Range r("sdirt_calib_fma64");
    return calib_fma64(n_threads, iters, out, (hipStream_t)stream);
}

}  // extern "C"
