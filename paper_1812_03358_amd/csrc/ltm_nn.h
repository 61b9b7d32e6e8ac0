// Descriptors shared by the warm-start network kernels and their C ABI.
#pragma once

#include "ltm_internal.h"

namespace ltm {

struct ConvFwd {
    const unsigned short* in0;
    const unsigned short* in1;
    int c0, c1;
    const unsigned short* wt;   // [rows][Kp] BF16, rows = 16 * (power of two >= cout/16)
    int Kp;
    const float* bias;
    void* out;
    void* out2;
    int cout, split, relu, out_f32, up;
    int D, H, W;                // output grid; input grid = output >> up
};

struct ConvWgrad {
    const unsigned short* in0;
    const unsigned short* in1;
    int c0, c1;
    const unsigned short* dy;   // [D*H*W][cout] BF16
    float* dw;                  // [cout][K] FP32, accumulated
    int cout, K, up;
    int D, H, W;
};

int nn_rows(int cout);          // padded row count of a packed weight matrix
int nn_kp(int k);               // K padded to a multiple of 32

hipError_t nn_conv_fwd(const ConvFwd& a, int ks, hipStream_t s);
hipError_t nn_conv_wgrad(const ConvWgrad& a, int ks, hipStream_t s);
hipError_t nn_pack(const float* w, int cout, int cin, int taps, unsigned short* wf, int rows_f, int kp_f,
                   unsigned short* wb, int rows_b, int kp_b, hipStream_t s);
hipError_t nn_maxpool(const unsigned short* x, unsigned short* y, unsigned char* arg, int D, int H, int W, int C,
                      hipStream_t s);
hipError_t nn_maxpool_bwd(const float* dy, const unsigned char* arg, float* dx, int D, int H, int W, int C,
                          hipStream_t s);
hipError_t nn_sumpool(const float* dh, float* dl, int D, int H, int W, int C, int accumulate, hipStream_t s);
hipError_t nn_relu_mask(const float* dout, const unsigned short* out, int relu, unsigned short* g,
                        float* dbias, size_t n, int C, hipStream_t s);
hipError_t nn_mse(const float* x, const float* t, float* g, double* loss, size_t n, hipStream_t s);
hipError_t nn_adam(float* w, float* g, float* m, float* v, size_t n, float lr, float b1, float b2, float eps,
                   int step, hipStream_t s);
hipError_t nn_prep_input(const float* x, unsigned short* y, unsigned int* scratch, size_t n, hipStream_t s);
hipError_t nn_add(float* a, const float* b, size_t n, hipStream_t s);

}  // namespace ltm
