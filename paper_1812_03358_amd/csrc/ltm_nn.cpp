// C ABI of the warm-start network building blocks: argument validation and
// launches (no allocation, asynchronous on the caller's stream).
#include <string>

#include "ltm_nn.h"

namespace ltm {

int nn_rows(int cout)
{
    const int nt = (cout + 15) / 16;
    return 16 * (nt <= 1 ? 1 : (nt <= 2 ? 2 : (nt <= 4 ? 4 : 8)));
}

int nn_kp(int k) { return (k + 31) / 32 * 32; }

namespace {

ltm_status check_conv(const ltm_nn_conv* c)
{
    if (!c) return fail(LTM_ERR_INVALID, "null descriptor");
    if (c->ksize != 1 && c->ksize != 3) return fail(LTM_ERR_INVALID, "ksize must be 1 or 3");
    if (c->d == 0 || c->h == 0 || c->w == 0) return fail(LTM_ERR_INVALID, "empty grid");
    if ((uint64_t)c->d * c->h * c->w >= (1ull << 31)) return fail(LTM_ERR_INVALID, "grid too large");
    if (c->upsample > 1) return fail(LTM_ERR_INVALID, "upsample must be 0 or 1");
    if (c->upsample && (c->d % 2 || c->h % 2 || c->w % 2))
        return fail(LTM_ERR_INVALID, "upsampling needs an even output grid");
    const uint32_t cin = c->c0 + c->c1;
    if (cin == 0 || c->cout == 0 || c->cout > 128) return fail(LTM_ERR_INVALID, "need 1 <= cout <= 128, cin >= 1");
    if (cin > 1 && (c->c0 % 8 || c->c1 % 8))
        return fail(LTM_ERR_INVALID, "input channel counts must be multiples of 8 (or a single channel)");
    if (cin == 1 && c->c1 != 0) return fail(LTM_ERR_INVALID, "a single input channel comes from in0");
    if (c->split == 0 || c->split > c->cout) return fail(LTM_ERR_INVALID, "split must be in [1, cout]");
    if (cin * c->ksize * c->ksize * c->ksize > 8192) return fail(LTM_ERR_INVALID, "reduction too long");
    return LTM_OK;
}

}  // namespace
}  // namespace ltm

using namespace ltm;

extern "C" {

ltm_status ltm_nn_packed_sizes(uint32_t cout, uint32_t cin, uint32_t ksize, uint64_t* fwd_elems,
                               uint64_t* bwd_elems)
{
    if (!fwd_elems || !bwd_elems) return fail(LTM_ERR_INVALID, "null argument");
    if ((ksize != 1 && ksize != 3) || cout == 0 || cin == 0 || cout > 128 || cin > 128)
        return fail(LTM_ERR_INVALID, "bad layer shape");
    const int taps = (int)(ksize * ksize * ksize);
    *fwd_elems = (uint64_t)nn_rows((int)cout) * nn_kp(taps * (int)cin);
    *bwd_elems = (uint64_t)nn_rows((int)cin) * nn_kp(taps * (int)cout);
    return LTM_OK;
}

ltm_status ltm_nn_pack_weights(const float* w, uint32_t cout, uint32_t cin, uint32_t ksize, uint16_t* w_fwd,
                               uint16_t* w_bwd, void* stream)
{
    uint64_t nf, nb;
    ltm_status st = ltm_nn_packed_sizes(cout, cin, ksize, &nf, &nb);
    if (st != LTM_OK) return st;
    if (!w || !w_fwd) return fail(LTM_ERR_INVALID, "null argument");
    const int taps = (int)(ksize * ksize * ksize);
    hipError_t e = nn_pack(w, (int)cout, (int)cin, taps, w_fwd, nn_rows((int)cout), nn_kp(taps * (int)cin),
                           w_bwd, nn_rows((int)cin), nn_kp(taps * (int)cout), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "pack weights");
    return LTM_OK;
}

ltm_status ltm_nn_conv3d_forward(const ltm_nn_conv* c, const uint16_t* in0, const uint16_t* in1,
                                 const uint16_t* w_fwd, const float* bias, void* out, void* out2, void* stream)
{
    ltm_status st = check_conv(c);
    if (st != LTM_OK) return st;
    if (!in0 || !w_fwd || !out || (c->c1 && !in1) || (c->split < c->cout && !out2))
        return fail(LTM_ERR_INVALID, "null buffer");
    ConvFwd a{};
    a.in0 = in0;
    a.in1 = in1;
    a.c0 = (int)c->c0;
    a.c1 = (int)c->c1;
    a.wt = w_fwd;
    a.Kp = nn_kp((int)(c->ksize * c->ksize * c->ksize * (c->c0 + c->c1)));
    a.bias = bias;
    a.out = out;
    a.out2 = out2;
    a.cout = (int)c->cout;
    a.split = (int)c->split;
    a.relu = c->relu ? 1 : 0;
    a.out_f32 = c->out_f32 ? 1 : 0;
    a.up = c->upsample ? 1 : 0;
    a.D = (int)c->d;
    a.H = (int)c->h;
    a.W = (int)c->w;
    hipError_t e = nn_conv_fwd(a, (int)c->ksize, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "conv3d forward");
    return LTM_OK;
}

ltm_status ltm_nn_conv3d_dgrad(const ltm_nn_conv* c, const uint16_t* dy, const uint16_t* w_bwd, float* dx0,
                               float* dx1, void* stream)
{
    ltm_status st = check_conv(c);
    if (st != LTM_OK) return st;
    if (c->cout % 8 && c->cout != 1) return fail(LTM_ERR_INVALID, "cout must be a multiple of 8 for dgrad");
    if (!dy || !w_bwd || !dx0 || (c->c1 && !dx1)) return fail(LTM_ERR_INVALID, "null buffer");
    ltm_nn_conv t{};
    t.ksize = c->ksize;
    t.d = c->d;
    t.h = c->h;
    t.w = c->w;
    t.c0 = c->cout;
    t.c1 = 0;
    t.cout = c->c0 + c->c1;
    t.split = c->c1 ? c->c0 : t.cout;
    t.relu = 0;
    t.out_f32 = 1;
    t.upsample = 0;
    return ltm_nn_conv3d_forward(&t, dy, nullptr, w_bwd, nullptr, dx0, dx1, stream);
}

ltm_status ltm_nn_conv3d_wgrad(const ltm_nn_conv* c, const uint16_t* in0, const uint16_t* in1, const uint16_t* dy,
                               float* dw, void* stream)
{
    ltm_status st = check_conv(c);
    if (st != LTM_OK) return st;
    if (!in0 || !dy || !dw || (c->c1 && !in1)) return fail(LTM_ERR_INVALID, "null buffer");
    ConvWgrad a{};
    a.in0 = in0;
    a.in1 = in1;
    a.c0 = (int)c->c0;
    a.c1 = (int)c->c1;
    a.dy = dy;
    a.dw = dw;
    a.cout = (int)c->cout;
    a.K = (int)(c->ksize * c->ksize * c->ksize * (c->c0 + c->c1));
    a.up = c->upsample ? 1 : 0;
    a.D = (int)c->d;
    a.H = (int)c->h;
    a.W = (int)c->w;
    hipError_t e = nn_conv_wgrad(a, (int)c->ksize, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "conv3d wgrad");
    return LTM_OK;
}

ltm_status ltm_nn_maxpool2(const uint16_t* x, uint16_t* y, uint8_t* arg, uint32_t d, uint32_t h, uint32_t w,
                           uint32_t c, void* stream)
{
    if (!x || !y || !arg || c == 0 || d % 2 || h % 2 || w % 2 || d == 0)
        return fail(LTM_ERR_INVALID, "maxpool needs an even non-empty grid");
    hipError_t e = nn_maxpool(x, y, arg, (int)d, (int)h, (int)w, (int)c, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "maxpool");
    return LTM_OK;
}

ltm_status ltm_nn_maxpool2_backward(const float* dy, const uint8_t* arg, float* dx, uint32_t d, uint32_t h,
                                    uint32_t w, uint32_t c, void* stream)
{
    if (!dy || !arg || !dx || c == 0 || d % 2 || h % 2 || w % 2 || d == 0)
        return fail(LTM_ERR_INVALID, "maxpool needs an even non-empty grid");
    hipError_t e = nn_maxpool_bwd(dy, arg, dx, (int)d, (int)h, (int)w, (int)c, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "maxpool backward");
    return LTM_OK;
}

ltm_status ltm_nn_upsample2_backward(const float* d_high, float* d_low, uint32_t d, uint32_t h, uint32_t w,
                                     uint32_t c, uint32_t accumulate, void* stream)
{
    if (!d_high || !d_low || c == 0 || d % 2 || h % 2 || w % 2 || d == 0)
        return fail(LTM_ERR_INVALID, "upsampling needs an even non-empty grid");
    hipError_t e = nn_sumpool(d_high, d_low, (int)d, (int)h, (int)w, (int)c, accumulate ? 1 : 0,
                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "upsample backward");
    return LTM_OK;
}

ltm_status ltm_nn_relu_backward(const float* d_out, const uint16_t* out, uint32_t relu, uint16_t* g,
                                float* d_bias, uint64_t n, uint32_t c, void* stream)
{
    if (!d_out || !g || (relu && !out) || c == 0 || c > 1024 || n % c)
        return fail(LTM_ERR_INVALID, "bad relu backward arguments");
    hipError_t e = nn_relu_mask(d_out, out, relu ? 1 : 0, g, d_bias, n, (int)c, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "relu backward");
    return LTM_OK;
}

ltm_status ltm_nn_mse(const float* x, const float* target, float* grad, double* loss, uint64_t n, void* stream)
{
    if (!x || !target || !grad || !loss || n == 0) return fail(LTM_ERR_INVALID, "null argument");
    hipError_t e = nn_mse(x, target, grad, loss, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "mse");
    return LTM_OK;
}

ltm_status ltm_nn_adam(float* w, float* g, float* m, float* v, uint64_t n, double lr, double beta1, double beta2,
                       double eps, uint32_t step, void* stream)
{
    if (!w || !g || !m || !v || n == 0 || step == 0) return fail(LTM_ERR_INVALID, "bad Adam arguments");
    hipError_t e = nn_adam(w, g, m, v, n, (float)lr, (float)beta1, (float)beta2, (float)eps, (int)step,
                           static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "adam");
    return LTM_OK;
}

ltm_status ltm_nn_prep_input(const float* x, uint16_t* y, uint32_t* scratch, uint64_t n, void* stream)
{
    if (!x || !y || !scratch || n == 0) return fail(LTM_ERR_INVALID, "null argument");
    hipError_t e = nn_prep_input(x, y, scratch, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "prep input");
    return LTM_OK;
}

ltm_status ltm_nn_add(float* a, const float* b, uint64_t n, void* stream)
{
    if (!a || !b) return fail(LTM_ERR_INVALID, "null argument");
    hipError_t e = nn_add(a, b, n, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "add");
    return LTM_OK;
}

}  // extern "C"
