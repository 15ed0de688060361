// unet.h -- device runtime of the 3-D convolutional U-Net surrogate that
// predicts a temperature field from a density field (the learned starting
// point for the plain iteration; it stands where the paper starts the
// iteration from a reference field, Sec. 2.1.2).
//
// Architecture (channels-last, BF16 activations, FP32 accumulation and
// FP32 master weights): `levels` resolution levels with base * 2^l
// channels; each level has two 3^3 convolutions (zero padding) followed by
// a leaky ReLU of slope 0.1; a stride-2 2^3 convolution (+ leaky ReLU) goes
// down, a stride-2 transposed 2^3 convolution (+ leaky ReLU) comes up and is
// concatenated after the skip tensor of the level; a final 3^3 convolution
// without activation produces `cout` channels.
//
// Parameters live in one FP32 array, layer by layer in the order
//   e0a e0b d0 e1a e1b d1 ... e{L-1}a e{L-1}b u{L-2} q{L-2}a q{L-2}b ... u0 q0a q0b out
// each layer as weights w[kz][ky][kx][cin][cout] followed by biases b[cout].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace soc {
namespace unet {

struct View {   // channels-last BF16 tensor view: element (pos, c) at p[pos * cs + co + c]
    uint16_t *p = nullptr;
    int32_t cs = 0, co = 0, c = 0;
    View at(int32_t off, int32_t n) const { return View{p, cs, co + off, n}; }
};

struct Layer {
    enum Kind { CONV3, DOWN2, UP2 } kind;
    std::string name;
    int32_t cin = 0, cout = 0;       // real channel counts
    int32_t cin_buf = 0;             // channels of the input view (multiple of 16; >= cin)
    int32_t cout_buf = 0;            // channels of the gradient view fed to the backward-data pass
    int32_t level_in = 0, level_out = 0;
    int64_t w_off = 0, b_off = 0;    // offsets in the parameter array
    int64_t nw = 0;
    uint16_t *wf = nullptr;          // forward weights, [phase][npad_f][taps * cin_buf]
    uint16_t *wb = nullptr;          // backward-data weights, [phase][npad_b][taps * cout_buf]
    int32_t npad_f = 0, npad_b = 0;
};

class Net {
public:
    enum Code { OK, BAD_SHAPE, NO_MEMORY, HIP_ERROR };
    struct Status {
        Code code;
        std::string msg;
    };
    // Allocates parameters (He-normal weights from the seed, zero biases),
    // optimiser state and every activation and gradient buffer for up to
    // nmax samples of nz x ny x nx cells.
    Status create(int device, int32_t cin, int32_t cout, int32_t base, int32_t levels, int32_t nmax, int32_t nz,
                  int32_t ny, int32_t nx, uint64_t seed, hipStream_t s);
    void destroy();
    ~Net() { destroy(); }

    int64_t param_count() const { return nparam_; }
    hipError_t set_params(const float *h, hipStream_t s);
    hipError_t get_params(float *h, hipStream_t s);
    hipError_t get_grads(float *h, hipStream_t s);
    // x: device FP32 [n][nz][ny][nx][cin]; y: device FP32 [n][nz][ny][nx][cout]
    hipError_t forward(int32_t n, const float *d_x, float *d_y, hipStream_t s);
    // Gradients of sum(dy * y) for the last forward, into the FP32 gradient array.
    // stop_layer >= 0 (test hook): return once that layer (parameter order)
    // has its weight gradient and, where it has one, its backward-data
    // result, so that the tensors it consumed and produced are still intact.
    hipError_t backward(const float *d_dy, hipStream_t s, int32_t stop_layer = -1);
    // Test hook: copy one stored BF16 tensor of a layer (parameter order) to
    // host FP32, real channels only, [n][positions][channels] for the batch
    // of the last forward.  which: 0 the forward input, 1 the forward output
    // (not stored for the last layer, whose output is the caller's FP32
    // array), 2 the output-side gradient its weight gradient and
    // backward-data pass consumed in the last backward, 3 its backward-data
    // result (slope and skip gradient applied).  BAD_SHAPE when the tensor
    // does not exist or count differs; 2 and 3 hold only for the layer a
    // backward stopped at.
    Status read(int32_t layer, int32_t which, float *h, int64_t count, hipStream_t s);
    int32_t layer_count() const { return (int32_t)layers_.size(); }
    // Mean squared error of y against t over n samples (host FP64 result
    // when h_loss is non-NULL; synchronises), and its gradient into d_dy.
    hipError_t mse(int32_t n, const float *d_y, const float *d_t, float *d_dy, double *h_loss, hipStream_t s);
    hipError_t adam(float lr, float beta1, float beta2, float eps, int32_t step, hipStream_t s);
    hipError_t zero_grads(hipStream_t s);
    int64_t flops_forward(int32_t n) const;   // multiply-adds x 2 of the real (unpadded) network

    int device = 0;
    int32_t cin_ = 0, cout_ = 0, base_ = 0, levels_ = 0, nmax_ = 0, nz_ = 0, ny_ = 0, nx_ = 0;
    int32_t n_last_ = 0;   // batch of the last forward

private:
    hipError_t prep_weights(hipStream_t s);
    hipError_t conv_fwd(const Layer &L, int32_t n, const View &x, const View &y, float *yf, int32_t yf_cs,
                        hipStream_t s);
    hipError_t conv_bwd_data(const Layer &L, int32_t n, const View &dy, const View &slope, const View *add,
                             const View &dx, hipStream_t s);
    hipError_t conv_wgrad(const Layer &L, int32_t n, const View &x, const View &dy, hipStream_t s);
    struct WgradPlan {
        int64_t chunks = 0;
        uint32_t chunk = 0;   // bricks (3^3 layers) or rows per chunk
        bool bricks = false;
    };
    WgradPlan plan_wgrad(const Layer &L, int32_t n) const;
    int64_t positions(int level, int32_t n) const;

    std::vector<Layer> layers_;
    // views each layer used in the last forward / backward (read hook)
    std::vector<View> fin_, fout_, bdy_, bdx_;
    int64_t nparam_ = 0;
    float *d_params_ = nullptr, *d_grads_ = nullptr, *d_m_ = nullptr, *d_v_ = nullptr;
    float *d_part_ = nullptr;   // split-K weight-gradient partials
    int64_t cap_part_ = 0;
    void *d_prep_ = nullptr;    // the weight-layout jobs of every layer (device table)
    int32_t n_prep_ = 0;
    int64_t max_prep_ = 0;      // elements of the largest job
    double *d_loss_part_ = nullptr;
    uint16_t *d_xin_ = nullptr;   // padded BF16 input
    uint16_t *d_gy_ = nullptr;    // padded BF16 output gradient
    int32_t cin_pad_ = 0, cout_pad_ = 0;
    std::vector<uint16_t *> ha_, cat_, hd_, hqa_, hqb_, g1_, g2_, gcat_;
    uint16_t *hbot_ = nullptr;
    std::vector<void *> allocs_;
};

}  // namespace unet
}  // namespace soc
