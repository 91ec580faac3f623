// Learned correction of the multigrid preconditioner: a 6-layer residual CNN
// (3x3 convolutions, 32 channels) on the nodal grid, with BF16 weights and
// activations on the matrix cores and FP32 accumulation, trained on the device
// with Adam.
//
//   h0 = relu(conv(x) + b0)                    3 -> 32 channels
//   h_l = h_{l-1} + relu(conv(h_{l-1}) + b_l)   l = 1..4
//   y = conv(h4) + b5                          32 -> 1 channel
//
// Parameters are packed per layer as W[c_out][c_in][3][3] then b[c_out]
// (FP32 master copy); the kernels use BF16 copies padded to 16 / 32 channels.
// Activations are stored pixel-major with channels innermost.
#pragma once

#include "common.h"

namespace hinv {

class Cnn {
  public:
    static constexpr int kLayers = 6;
    static constexpr int kCh = 32;    // hidden channels
    static constexpr int kInCh = 3;   // residual, log-coefficient, free-node mask
    static constexpr int kPadIn = 16;  // input / output channels padded to one MFMA K-step
    explicit Cnn(Ctx* ctx);

    static int nparams();
    void set_params(const float* host);
    void get_params(float* host) const;
    void reset_adam() { step_ = 0; }

    // Planar FP32 device images: in [B][3][S][S], out / target [B][S][S].
    void forward(int B, int S, const float* in, float* out);
    // Loss and its gradient (left on the device; copied to grad_host when
    // given).  tchan = 1: target [B][S][S], mean relative L2.  tchan = 4:
    // target [B][4][S][S] = (t, wE, wN, diag), mean relative energy norm
    // (y - t)^T A (y - t) / t^T A t on the free nodes (input channel 2) with A
    // the 5-point stencil of those weights.
    double gradient(int B, int S, const float* in, const float* target, int tchan, float* grad_host);
    // gradient + one Adam step (lr); returns the loss before the step.
    double train_step(int B, int S, const float* in, const float* target, int tchan, float lr);

    // Pre-packed path for the solver: the input buffer (bf16, 16 channels)
    // for one S x S image, the network run on it, and its FP32 output
    // (16 channels, channel 0 meaningful).
    short* packed_input(int S);
    void forward_packed(int B, int S);
    const float* packed_output() const { return z_[kLayers - 1].get(); }

  private:
    void ensure(int B, int S);
    void refresh_weights();
    void run_forward(int B, int S);

    Ctx* ctx_;
    DBuf<float> theta_, grad_, m_, v_;
    int step_ = 0;
    bool weights_fresh_ = false;
    DBuf<short> wf_[kLayers], wb_[kLayers];  // forward [9][co][ci], backward [9][ci][co] (flipped)
    DBuf<short> in0_, a_[kLayers - 1], dz_[2], gy_;
    DBuf<float> z_[kLayers], h_[kLayers - 1], gh_[2], part_, loss_;
    DBuf<double> lpart_, ratio_, dwtmp_;
    int B_ = 0, S_ = 0, nwg_ = 0;
};

}  // namespace hinv
