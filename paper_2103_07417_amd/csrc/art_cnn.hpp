// art_cnn.hpp -- learned refinement proposal network (internal).
//
// A batch holds B level-l vertex grids of H x W positions.  Interfaces
// (features, logits, labels) are NCHW FP32/uint8 ([b][c][y][x]); activations
// and their gradients are NHWC BF16 inside the network.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "art_internal.hpp"

namespace art {

constexpr int kCnnOut = 15;             // 3 points at level l+1, 12 at level l+2 per level-l vertex
constexpr int kCnnIn = 3;               // log intensity, minimum radius, equatorial crossings
constexpr int8_t kMarkPropose = 100;    // level map: point proposed for tracing
constexpr int8_t kMarkSuppress = 101;   // level map: point the network rejects
constexpr int8_t kMarkUnset = -2;       // level map before a learned render decides a point

// Convolution 3x3, zero padding, implicit GEMM on BF16 MFMA.  Input NHWC
// [B][H][W][cin_pad] BF16, Wm = packed forward matrix [32][9 * cin_pad].
// mode 0: out bf16 NHWC32 = relu(conv + b); mode 1: out f32 NCHW [B][co][H][W]
// = conv + b; mode 2: out bf16 NHWC32 = conv * (mask > 0), no bias (input
// gradient through a ReLU).  Returns hipErrorInvalidValue unless cin_pad is
// 8, 16, 24 or 32, Kp == 9 * cin_pad and 1 <= co <= 32.
hipError_t cnn_conv_fwd(const uint16_t* in, int cin_pad, int B, int H, int W, const uint16_t* Wm, int Kp,
                        const float* bias, int co, int mode, void* out, const uint16_t* mask,
                        hipStream_t s);
// Weight and bias gradients of a convolution: dW[co][ci][3][3] (FP32, master
// order) = sum over positions of dZ x im2col(in); in NHWC cin_pad, dZ NHWC
// cout_pad.  part holds cnn_dw_part_floats(B*H*W, cin_pad) floats.
hipError_t cnn_conv_dw(const uint16_t* in, int ci, int cin_pad, int B, int H, int W, const uint16_t* dZ, int co,
                       int cout_pad, float* part, float* dW, float* db, hipStream_t s);
long long cnn_dw_part_floats(long long positions, int cin_pad);
// FP32 master W[co][ci][3][3] -> BF16 forward matrix Wf[32][9 cin_pad] and
// (if Wb != NULL) input-gradient matrix Wb[32][9 cout_pad].
hipError_t cnn_pack(const float* Wt, int ci, int co, int cin_pad, int cout_pad, uint16_t* Wf, uint16_t* Wb,
                    hipStream_t s);
hipError_t cnn_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                    float eps, int t, hipStream_t s);
// Loss over B images: logits/labels/valid NCHW [B][15][HW]; dz NHWC [B][HW][16].
hipError_t cnn_bce(const float* z, const uint8_t* y, const uint8_t* valid, long long B, long long HW,
                   float pos_w, const float* inv_dev, uint16_t* dz, float* part, int nblocks, hipStream_t s);
// 1 / (number of nonzero valid[i], at least 1) into *inv_out; part holds nb counts.
hipError_t cnn_count_valid(const uint8_t* valid, long long n, unsigned long long* part, int nb, float* inv_out,
                           hipStream_t s);
// FP32 NCHW [B][3][HW] -> BF16 NHWC [B][HW][8].
hipError_t cnn_input_bf16(const float* x, long long B, long long HW, uint16_t* y, hipStream_t s);

// Features of one image's level-l vertex grid (H x W, stride s on the final
// grid of width nx) into x[3][H][W] (FP32).
hipError_t cnn_features(const double* img, const RayFeat* feat, long long nx, int s, int H, int W,
                        double nabs, float* x, hipStream_t st);
// Same for images of a batch: x[b][3][H][W] for image imap[b] (b < nimg; all
// images in order if imap is null), N_abs from the counters; with x null the
// network's BF16 input xb[b][H][W][8] instead (cnn_input_bf16's rounding).
hipError_t cnn_features_batch(const ImageDesc* desc, const Counters* ctr, int nimg, int l, int H, int W,
                              float* x, uint16_t* xb, hipStream_t st, const int* imap = nullptr);
// Labels of one plain render's level map at level l: lab/val[15][H][W].
hipError_t cnn_labels(const int8_t* level, long long nx, int nx0, int ny0, int N, int l, uint8_t* lab,
                      uint8_t* val, hipStream_t s);
// Proposals of every image from logits[b][15][H][W]: level-(l+1) points above
// z_hi are marked kMarkPropose, level-(l+2) points above z_hi are marked l+2
// and appended to the trace list of pass l+1 (of capacity cap: at the front
// when the largest step count of their cell's level-l corners reaches
// long_steps, else from the back); points below z_lo are marked
// kMarkSuppress, all others kMarkUnset (every owned point is written).  An
// image whose level count is l + 1 gets kMarkUnset everywhere unless
// all_levels (the plain criterion decides its last level).
// logits[b] belongs to image imap[b] (all images in order if imap is null).
hipError_t cnn_propose(const float* logits, const ImageDesc* desc, int nimg, int l, int H, int W,
                       float z_hi, float z_lo, int all_levels, unsigned long long* list, long long cap,
                       int long_steps, Counters* ctr, hipStream_t s, const int* imap = nullptr);

// Activation workspace of one forward pass over P = B * H * W positions.
struct CnnWork {
    long long cap = 0;         // positions the buffers hold
    uint16_t* x = nullptr;     // input [B][H][W][8] bf16
    uint16_t* act[3] = {};     // post-ReLU activations [B][H][W][32]
    float* logits = nullptr;   // [B][15][H][W]
};

// Network state (device): FP32 master parameters in the flat order
// W0, b0, W1, b1, W2, b2, W3, b3 (W[l] as [c_out][c_in][3][3]), Adam moments,
// packed BF16 matrices, workspaces.
struct CnnNet {
    int ci[4] = { kCnnIn, 32, 32, 32 };
    int co[4] = { 32, 32, 32, kCnnOut };
    int cin_pad[4] = { 8, 32, 32, 32 };       // NHWC channel padding of each layer's input
    int cout_pad[4] = { 32, 32, 32, 16 };     // ... and of its output gradient
    long long off_w[4] = {}, off_b[4] = {};
    int nparam = 0;
    float* p = nullptr;        // FP32 parameters
    float* g = nullptr;        // gradients
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    uint16_t* Wf[4] = {};      // forward matrices [32][9 cin_pad]
    uint16_t* Wb[4] = {};      // input-gradient matrices [32][9 cout_pad] (layers 1..3)
    int step = 0;
    CnnWork ws;                // workspace of the network's own calls
    uint16_t* dz0 = nullptr;   // gradient buffers [B][H][W][32]
    uint16_t* dz1 = nullptr;
    long long dz_cap = 0;
    float* part = nullptr;     // weight-gradient partials
    long long part_cap = 0;
    float* lossp = nullptr;    // loss partials [1024] + 1/n_valid
    unsigned long long* cntp = nullptr;   // valid-count partials [1024]
};

// Grow a workspace to P positions (synchronises the device when it grows).
int cnn_work_reserve(CnnWork* w, long long P);
void cnn_work_free(CnnWork* w);
// Logits of B feature grids x_dev [B][3][H][W] into logits [B][15][H][W]
// (x_dev null: the BF16 input is already in w->x).
hipError_t cnn_net_forward(const CnnNet* n, CnnWork* w, const float* x_dev, int B, int H, int W, float* logits,
                           hipStream_t s);

}  // namespace art

// Opaque handle of the C ABI.
struct art_cnn {
    art::CnnNet net;
};
