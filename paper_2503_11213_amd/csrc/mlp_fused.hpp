// Arguments of the fused surrogate inference kernels (width-256 networks),
// shared by the host code that fills them and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdirt {

typedef uint16_t bf16_t;

struct FusedArgs {
    long long n_rows;
    int n_hidden, n_out, n_freq, feat_pad;
    float x_half, y_half, iv_lo, iv_hi, lam_lo, lam_hi;
    const float* x;                 // [n_rows][4] (input rows)
    const float* params;            // float32 master (biases)
    long long b_off[17];            // bias offsets per layer
    const bf16_t* W[17];            // bf16 weights in matrix-core fragment order
    void* out;                      // [n_rows][n_out]
    int out_bf16;
    // Pixel rows (the fused surrogate render; depth != nullptr): row
    // ((n C + c) tiles + t) 64 + p is pixel p (row-major) of 8 x 8 tile t of
    // channel c of image n; its input is (h_x, h_y, 1 / depth, lam[c]).
    // Images: N = img_n, C = img_c, H = img_h, W = img_w.
    const float* depth;             // [N][H][W] (mm)
    const float* img;               // [N][C][H][W]
    float* rout;                    // [N][2C][H][W]
    int img_n, img_c, img_h, img_w, ks, tiles_x, tiles_y;
    float pitch;                    // mm per pixel
    float lam[4];                   // wavelength of each channel (um)
};

// Softmax inference of A.n_rows input rows into A.out, in chunks of `chunk`
// rows (hbuf: chunk x 256 bf16 of workspace).
int launch_mlp_fused(const FusedArgs& A, bf16_t* hbuf, long long chunk, hipStream_t st);
// The fused surrogate render of the pixel rows into A.rout.
int launch_mlp_render(const FusedArgs& A, bf16_t* hbuf, long long chunk, hipStream_t st);

}  // namespace sdirt
