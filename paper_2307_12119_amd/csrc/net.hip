// C ABI of the learned warm start: parameter storage, workspace plan and the host-side
// sequencing of the network's forward pass, its gradient and the Adam step.  Every operation
// is a kernel of nn.hip; the host only orders launches.
#include <cmath>
#include <vector>

#include "ctx.hpp"
#include "nn.hpp"

using namespace vs;

namespace {

struct NetLayer {
  int ks = 1, cin_src = 0, cin = 0, cout = 0;  // cin: padded input channels the kernels use
  long w_off = 0, b_off = 0;                   // offsets in the flat FP32 parameters
  size_t wb = 0, wt = 0;                       // element offsets of the BF16 copies (forward, transposed)
  int wblk = 0;                                // BF16 copies in the blocked layout (see w_index)
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

struct varsim_net {
  varsim_ctx* ctx = nullptr;
  varsim_net_config cfg{};
  long count = 0;
  float* p = nullptr;     // FP32 master parameters
  float* m = nullptr;     // Adam first moments
  float* v = nullptr;     // Adam second moments
  uint16_t* wbf = nullptr;
  size_t wbf_elems = 0;
  int adam_t = 0;
  NetLayer stem, enc[5][2], dec[4], head;
};

namespace {

int level_size(const varsim_net* net, int l) { return (net->cfg.n / 4) >> l; }

// Workspace plan of one batch: every buffer's byte offset (base = nullptr gives the size).
struct NetBufs {
  uint16_t *feat, *stem, *ea[5], *eb[5], *pool[5], *d[4];
  float* y;
  uint16_t *dh, *dz;
  float *mse_part, *dD, *dcat[4], *bufA, *bufX, *wpart, *rpart, *tmp;
  size_t total;
};

NetBufs plan(const varsim_net* net, int B, bool training, char* base) {
  NetBufs b{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += up256(bytes);
    return p;
  };
  const int* w = net->cfg.width;
  auto P = [&](int l) { return (size_t)B * level_size(net, l) * level_size(net, l); };
  b.feat = training ? (uint16_t*)take(P(0) * 64 * 2) : nullptr;
  b.stem = (uint16_t*)take(P(0) * w[0] * 2);
  for (int l = 0; l < 5; ++l) {
    if (l > 0) b.pool[l] = (uint16_t*)take(P(l) * w[l - 1] * 2);
    b.ea[l] = (uint16_t*)take(P(l) * w[l] * 2);
    b.eb[l] = (uint16_t*)take(P(l) * w[l] * 2);
  }
  for (int l = 0; l < 4; ++l) b.d[l] = (uint16_t*)take(P(l) * w[l] * 2);
  if (training) {
    const size_t n = net->cfg.n;
    b.y = (float*)take((size_t)B * n * n * 4);
    b.dh = (uint16_t*)take(P(0) * 16 * 2);
    size_t zmax = P(0) * 16, dmax = 0, xmax = 0;
    for (int l = 0; l < 5; ++l) {
      zmax = std::max(zmax, P(l) * w[l]);
      dmax = std::max(dmax, P(l) * w[l]);
      xmax = std::max(xmax, P(l) * (l ? w[l - 1] : w[0]));
    }
    b.dz = (uint16_t*)take(zmax * 2);
    b.mse_part = (float*)take(kNnMseBlocks * 17 * 4);
    b.dD = (float*)take(dmax * 4);
    // input gradient of each decoder layer, kept until the encoder has read its skip part
    for (int l = 0; l < 4; ++l) b.dcat[l] = (float*)take(P(l) * (w[l + 1] + w[l]) * 4);
    b.bufA = (float*)take(dmax * 4);
    b.bufX = (float*)take(xmax * 4);
    // largest weight-gradient partial buffer over the layers
    size_t wp = 0;
    auto wpl = [&](const NetLayer& L, int l) {
      const int m = level_size(net, l);
      wp = std::max(wp, (size_t)nn_wgrad_splits(L.ks, B, m, m, L.cin, L.cout) * L.cout * L.ks * L.ks * L.cin);
    };
    wpl(net->stem, 0);
    wpl(net->head, 0);
    for (int l = 0; l < 5; ++l) wpl(net->enc[l][0], l), wpl(net->enc[l][1], l);
    for (int l = 0; l < 4; ++l) wpl(net->dec[l], l);
    b.wpart = (float*)take(wp * 4);
    b.rpart = (float*)take((size_t)kNnReluBlocks * 256 * 4);
    b.tmp = (float*)take(64 * 4);
  }
  b.total = off;
  return b;
}

varsim_status check_config(varsim_ctx* ctx, const varsim_net_config* c) {
  if (!c) return fail(ctx, VARSIM_ERR_INVALID, "config is NULL");
  if (c->n < 64 || c->n > 1024 || c->n % 64) return fail(ctx, VARSIM_ERR_UNSUPPORTED, "n must be a multiple of 64 in [64, 1024]");
  for (int l = 0; l < 5; ++l)
    if (c->width[l] < 16 || c->width[l] > 256 || c->width[l] % 16)
      return fail(ctx, VARSIM_ERR_UNSUPPORTED, "widths must be multiples of 16 in [16, 256]");
  if (c->width[3] + c->width[4] > 512) return fail(ctx, VARSIM_ERR_UNSUPPORTED, "decoder input too wide");
  if (!std::isfinite(c->out_scale) || !std::isfinite(c->k0_W_mK) || !(c->k0_W_mK > 0))
    return fail(ctx, VARSIM_ERR_INVALID, "out_scale must be finite and k0 positive");
  return VARSIM_OK;
}

// Parameter order of the flat vector (see the header) and the BF16 copy layout.
void build_layers(varsim_net* net) {
  const int* w = net->cfg.width;
  long off = 0;
  size_t bo = 0;
  // 3x3 layers keep their weights blocked: the A operands of a matrix-core step are then one
  // contiguous kilobyte
  auto add = [&](NetLayer& L, int ks, int cin_src, int cin, int cout) {
    L.wblk = ks == 3 ? 1 : 0;
    L.ks = ks, L.cin_src = cin_src, L.cin = cin, L.cout = cout;
    L.w_off = off;
    off += (long)cout * ks * ks * cin_src;
    L.b_off = off;
    off += cout;
    const size_t e = (size_t)cout * ks * ks * cin;
    L.wb = bo;
    bo += (e + 127) / 128 * 128;
    L.wt = bo;
    bo += (e + 127) / 128 * 128;
  };
  add(net->stem, 1, 48, 64, w[0]);
  for (int l = 0; l < 5; ++l) {
    const int cin = l == 0 ? w[0] : w[l - 1];
    add(net->enc[l][0], 3, cin, cin, w[l]);
    add(net->enc[l][1], 3, w[l], w[l], w[l]);
  }
  for (int l = 3; l >= 0; --l) add(net->dec[l], 3, w[l + 1] + w[l], w[l + 1] + w[l], w[l]);
  add(net->head, 1, w[0], w[0], 16);
  net->count = off;
  net->wbf_elems = bo;
}

template <class F>
void for_layers(varsim_net* net, F&& f) {
  f(net->stem);
  for (int l = 0; l < 5; ++l) f(net->enc[l][0]), f(net->enc[l][1]);
  for (int l = 3; l >= 0; --l) f(net->dec[l]);
  f(net->head);
}

hipError_t refresh_bf16(varsim_net* net, hipStream_t s) {
  hipError_t e = hipSuccess;
  for_layers(net, [&](const NetLayer& L) {
    if (e != hipSuccess) return;
    e = nn_weight_cast(net->p + L.w_off, L.cout, L.ks * L.ks, L.cin_src, L.cin, net->wbf + L.wb, net->wbf + L.wt, s,
                       L.wblk);
  });
  return e;
}

NnConv conv_args(const varsim_net* net, const NetLayer& L, const uint16_t* x, int cx, const uint16_t* xu, int cu,
                 void* y, int B, int l, bool with_bias) {
  NnConv a{};
  a.x = x, a.cx = cx, a.xu = xu, a.cu = cu;
  a.w = net->wbf + L.wb;
  a.wblk = L.wblk;
  a.bias = with_bias ? net->p + L.b_off : nullptr;
  a.y = y;
  a.B = B, a.H = a.W = level_size(net, l);
  a.cout = L.cout;
  a.out_scale = net->cfg.out_scale;
  return a;
}

// dgrad of layer L: dz [P][cout] -> out FP32 [P][cin]
NnConv dgrad_args(const varsim_net* net, const NetLayer& L, const uint16_t* dz, float* out, int B, int l) {
  NnConv a{};
  a.x = dz, a.cx = L.cout;
  a.w = net->wbf + L.wt;
  a.wblk = L.wblk;
  a.y = out;
  a.B = B, a.H = a.W = level_size(net, l);
  a.cout = L.cin;
  return a;
}

// timing classes of the forward pass, one per layer ("fwd:conv:*" are the convolutions)
const char* const kFwdEncA[5] = {"fwd:conv:enc0a", "fwd:conv:enc1a", "fwd:conv:enc2a", "fwd:conv:enc3a",
                                 "fwd:conv:enc4a"};
const char* const kFwdEncB[5] = {"fwd:conv:enc0b", "fwd:conv:enc1b", "fwd:conv:enc2b", "fwd:conv:enc3b",
                                 "fwd:conv:enc4b"};
const char* const kFwdDec[4] = {"fwd:conv:dec0", "fwd:conv:dec1", "fwd:conv:dec2", "fwd:conv:dec3"};
const char* const kFwdPool[5] = {"", "fwd:elem:pool1", "fwd:elem:pool2", "fwd:elem:pool3", "fwd:elem:pool4"};

// training: also keep the features and the last decoder output (the gradient pass reads them);
// inference fuses the head into the last decoder convolution.
varsim_status run_forward(varsim_net* net, int B, const float* q, const float* v, const float* m, const int* idx,
                          float* out, const NetBufs& b, bool training, hipStream_t s) {
  varsim_ctx* ctx = net->ctx;
  const int* w = net->cfg.width;
  NnFeat f;
  for (int c = 0; c < 3; ++c) f.shift[c] = net->cfg.shift[c], f.scale[c] = net->cfg.scale[c];
  f.k0 = net->cfg.k0_W_mK;
  HIP_TRY(timed(ctx, "fwd:conv:stem", s, [&] {
    return nn_stem(q, v, m, idx, net->cfg.n, B, f, net->wbf + net->stem.wb, net->p + net->stem.b_off, w[0], b.stem,
                   training ? b.feat : nullptr, s);
  }));
  for (int l = 0; l < 5; ++l) {
    const uint16_t* in = b.stem;
    int cin = w[0];
    if (l > 0) {
      const int ml = level_size(net, l);
      HIP_TRY(timed(ctx, kFwdPool[l], s, [&] { return nn_avgpool(b.eb[l - 1], b.pool[l], B, ml, ml, w[l - 1], s); }));
      in = b.pool[l];
      cin = w[l - 1];
    }
    HIP_TRY(timed(ctx, kFwdEncA[l], s, [&] {
      return nn_conv(3, NN_EPI_BF16, true, conv_args(net, net->enc[l][0], in, cin, nullptr, 0, b.ea[l], B, l, true), s);
    }));
    HIP_TRY(timed(ctx, kFwdEncB[l], s, [&] {
      return nn_conv(3, NN_EPI_BF16, true, conv_args(net, net->enc[l][1], b.ea[l], w[l], nullptr, 0, b.eb[l], B, l, true),
                     s);
    }));
  }
  for (int l = 3; l >= 0; --l) {
    const uint16_t* up = l == 3 ? b.eb[4] : b.d[l + 1];
    if (l == 0 && !training && w[0] == 32) {  // last decoder layer with the head in its epilogue
      NnConv a = conv_args(net, net->dec[0], b.eb[0], w[0], up, w[1], out, B, 0, true);
      a.w2 = net->wbf + net->head.wb;
      a.bias2 = net->p + net->head.b_off;
      HIP_TRY(timed(ctx, "fwd:conv:dec0+head", s, [&] { return nn_conv(3, NN_EPI_HEAD, true, a, s); }));
      return VARSIM_OK;
    }
    HIP_TRY(timed(ctx, kFwdDec[l], s, [&] {
      return nn_conv(3, NN_EPI_BF16, true, conv_args(net, net->dec[l], b.eb[l], w[l], up, w[l + 1], b.d[l], B, l, true),
                     s);
    }));
  }
  HIP_TRY(timed(ctx, "fwd:conv:head", s, [&] {
    return nn_conv(1, NN_EPI_SHUFFLE, false, conv_args(net, net->head, b.d[0], w[0], nullptr, 0, out, B, 0, true), s);
  }));
  return VARSIM_OK;
}

// weight and bias gradient of layer L at level l: x / xu its input sources, dz its output gradient
varsim_status layer_wgrad(varsim_net* net, const NetLayer& L, const uint16_t* x, int cx, const uint16_t* xu, int cu,
                          const uint16_t* dz, int B, int l, float* grad, const NetBufs& b, hipStream_t s) {
  varsim_ctx* ctx = net->ctx;
  NnConv a = conv_args(net, L, x, cx, xu, cu, nullptr, B, l, false);
  const int m = level_size(net, l);
  const int ns = nn_wgrad_splits(L.ks, B, m, m, a.cu + a.cx, L.cout);
  HIP_TRY(timed(ctx, "nn_wgrad", s, [&] { return nn_wgrad(L.ks, a, dz, b.wpart, ns, s); }));
  HIP_TRY(timed(ctx, "nn_reduce", s, [&] {
    return nn_reduce_parts(b.wpart, ns, L.cout, L.ks * L.ks, L.cin, L.cin_src, grad + L.w_off, s);
  }));
  return VARSIM_OK;
}

// Gradient sources of a ReLU output at level l (C channels): da on the same grid (lda floats per
// pixel), dfine on the grid of level l - 1 (ldf floats per pixel; the gradient through the
// upsampling into the finer decoder), dpool on level l + 1 (the gradient through the pooling into
// the coarser encoder).
struct GradIn {
  const float* da = nullptr;
  int lda = 0;
  const float* dfine = nullptr;
  int ldf = 0;
  const float* dpool = nullptr;
};

varsim_status relu_back(varsim_net* net, const GradIn& g, const uint16_t* act, int B, int l, int C, float* bias_grad,
                        const NetBufs& b, hipStream_t s) {
  varsim_ctx* ctx = net->ctx;
  const int ml = level_size(net, l);
  HIP_TRY(timed(ctx, "nn_elementwise", s, [&] {
    return nn_relu_bwd(g.da, g.lda, g.dfine, g.ldf, g.dpool, act, b.dz, B, ml, ml, C, b.rpart, s);
  }));
  HIP_TRY(timed(ctx, "nn_reduce", s, [&] { return nn_colsum(b.rpart, kNnReluBlocks, C, C, 1.f, bias_grad, s); }));
  return VARSIM_OK;
}

varsim_status run_gradient(varsim_net* net, int B, const int* idx, const float* target, float* grad, float* loss,
                           const NetBufs& b, hipStream_t s) {
  varsim_ctx* ctx = net->ctx;
  const int* w = net->cfg.width;
  const int n = net->cfg.n;
  varsim_status st;
  // loss, head
  HIP_TRY(timed(ctx, "nn_elementwise", s,
                [&] { return nn_mse_grad(b.y, target, idx, n, B, net->cfg.out_scale, b.dh, b.mse_part, s); }));
  HIP_TRY(timed(ctx, "nn_reduce", s, [&] {
    return nn_colsum(b.mse_part, kNnMseBlocks, 17, 16, 1.f, grad + net->head.b_off, s);
  }));
  const float inv = (float)(1.0 / ((double)B * n * n));
  HIP_TRY(timed(ctx, "nn_reduce", s, [&] { return nn_colsum(b.mse_part + 16, kNnMseBlocks, 17, 1, inv, loss, s); }));
  if ((st = layer_wgrad(net, net->head, b.d[0], w[0], nullptr, 0, b.dh, B, 0, grad, b, s)) != VARSIM_OK) return st;
  HIP_TRY(timed(ctx, "nn_conv_dgrad", s,
                [&] { return nn_conv(1, NN_EPI_F32, false, dgrad_args(net, net->head, b.dh, b.dD, B, 0), s); }));
  // decoder, level 0 first.  dcat[l] = gradient of dec l's input [upsampled d_{l+1} | e_l]; the
  // gradient of d_l is dD (from the head) at level 0, else the sum over 2 x 2 blocks of the
  // upsampled part of dcat[l - 1]; d_4 is e_4
  for (int l = 0; l < 4; ++l) {
    const NetLayer& L = net->dec[l];
    GradIn g;
    if (l == 0)
      g.da = b.dD, g.lda = w[0];
    else
      g.dfine = b.dcat[l - 1], g.ldf = w[l] + w[l - 1];
    if ((st = relu_back(net, g, b.d[l], B, l, w[l], grad + L.b_off, b, s)) != VARSIM_OK) return st;
    const uint16_t* up = l == 3 ? b.eb[4] : b.d[l + 1];
    if ((st = layer_wgrad(net, L, b.eb[l], w[l], up, w[l + 1], b.dz, B, l, grad, b, s)) != VARSIM_OK) return st;
    HIP_TRY(timed(ctx, "nn_conv_dgrad", s,
                  [&] { return nn_conv(3, NN_EPI_F32, false, dgrad_args(net, L, b.dz, b.dcat[l], B, l), s); }));
  }
  // encoder, deepest level first: gradient of e_l = skip part of dcat[l] + pooled part from level
  // l + 1 (level 4: the upsampled part of dcat[3])
  for (int l = 4; l >= 0; --l) {
    const NetLayer& La = net->enc[l][0];
    const NetLayer& Lb = net->enc[l][1];
    GradIn g;
    if (l == 4)
      g.dfine = b.dcat[3], g.ldf = w[4] + w[3];
    else
      g.da = b.dcat[l] + w[l + 1], g.lda = w[l + 1] + w[l], g.dpool = b.bufX;
    if ((st = relu_back(net, g, b.eb[l], B, l, w[l], grad + Lb.b_off, b, s)) != VARSIM_OK) return st;
    if ((st = layer_wgrad(net, Lb, b.ea[l], w[l], nullptr, 0, b.dz, B, l, grad, b, s)) != VARSIM_OK) return st;
    HIP_TRY(timed(ctx, "nn_conv_dgrad", s,
                  [&] { return nn_conv(3, NN_EPI_F32, false, dgrad_args(net, Lb, b.dz, b.bufA, B, l), s); }));
    GradIn ga;
    ga.da = b.bufA, ga.lda = w[l];
    if ((st = relu_back(net, ga, b.ea[l], B, l, w[l], grad + La.b_off, b, s)) != VARSIM_OK) return st;
    const uint16_t* in = l == 0 ? b.stem : b.pool[l];
    const int cin = l == 0 ? w[0] : w[l - 1];
    if ((st = layer_wgrad(net, La, in, cin, nullptr, 0, b.dz, B, l, grad, b, s)) != VARSIM_OK) return st;
    HIP_TRY(timed(ctx, "nn_conv_dgrad", s,
                  [&] { return nn_conv(3, NN_EPI_F32, false, dgrad_args(net, La, b.dz, b.bufX, B, l), s); }));
  }
  // stem (bufX: gradient of the stem output)
  GradIn gs;
  gs.da = b.bufX, gs.lda = w[0];
  if ((st = relu_back(net, gs, b.stem, B, 0, w[0], grad + net->stem.b_off, b, s)) != VARSIM_OK) return st;
  if ((st = layer_wgrad(net, net->stem, b.feat, 64, nullptr, 0, b.dz, B, 0, grad, b, s)) != VARSIM_OK) return st;
  return VARSIM_OK;
}

varsim_status check_batch(varsim_net* net, int batch, const float* q, void* ws, size_t ws_bytes, bool training) {
  varsim_ctx* ctx = net->ctx;
  if (batch < 1) return fail(ctx, VARSIM_ERR_INVALID, "batch must be >= 1");
  if (!q || !ws) return fail(ctx, VARSIM_ERR_INVALID, "q_dyn and workspace are required");
  const size_t need = plan(net, batch, training, nullptr).total;
  if (ws_bytes < need) return fail(ctx, VARSIM_ERR_NO_MEMORY, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  return VARSIM_OK;
}

}  // namespace

extern "C" {

varsim_status varsim_net_create(varsim_ctx* ctx, const varsim_net_config* cfg, varsim_net** out) {
  if (!ctx || !out) return VARSIM_ERR_INVALID;
  *out = nullptr;
  varsim_status st = check_config(ctx, cfg);
  if (st != VARSIM_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  varsim_net* net = new varsim_net();
  net->ctx = ctx;
  net->cfg = *cfg;
  build_layers(net);
  const size_t pb = net->count * sizeof(float);
  if (hipMalloc(&net->p, pb) != hipSuccess || hipMalloc(&net->m, pb) != hipSuccess ||
      hipMalloc(&net->v, pb) != hipSuccess || hipMalloc(&net->wbf, net->wbf_elems * 2) != hipSuccess) {
    varsim_net_destroy(net);
    return fail(ctx, VARSIM_ERR_NO_MEMORY, "network parameter allocation failed");
  }
  if (hipMemset(net->p, 0, pb) != hipSuccess || hipMemset(net->m, 0, pb) != hipSuccess ||
      hipMemset(net->v, 0, pb) != hipSuccess || hipMemset(net->wbf, 0, net->wbf_elems * 2) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    varsim_net_destroy(net);
    return fail(ctx, VARSIM_ERR_DEVICE, "network parameter initialisation failed");
  }
  *out = net;
  return VARSIM_OK;
}

void varsim_net_destroy(varsim_net* net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(net->p);
  (void)hipFree(net->m);
  (void)hipFree(net->v);
  (void)hipFree(net->wbf);
  delete net;
}

varsim_status varsim_net_param_count(const varsim_net* net, int64_t* count) {
  if (!net || !count) return VARSIM_ERR_INVALID;
  *count = net->count;
  return VARSIM_OK;
}

varsim_status varsim_net_set_params(varsim_net* net, const float* params, void* stream) {
  if (!net) return VARSIM_ERR_INVALID;
  varsim_ctx* ctx = net->ctx;
  if (!params) return fail(ctx, VARSIM_ERR_INVALID, "params is NULL");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t pb = net->count * sizeof(float);
  HIP_TRY(hipMemcpyAsync(net->p, params, pb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(launch_zero_words(net->m, pb, s));
  HIP_TRY(launch_zero_words(net->v, pb, s));
  net->adam_t = 0;
  HIP_TRY(refresh_bf16(net, s));
  return VARSIM_OK;
}

varsim_status varsim_net_get_params(varsim_net* net, float* params, void* stream) {
  if (!net) return VARSIM_ERR_INVALID;
  varsim_ctx* ctx = net->ctx;
  if (!params) return fail(ctx, VARSIM_ERR_INVALID, "params is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemcpyAsync(params, net->p, net->count * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return VARSIM_OK;
}

varsim_status varsim_net_workspace_size(varsim_net* net, int32_t batch, int32_t training, size_t* bytes) {
  if (!net || !bytes) return VARSIM_ERR_INVALID;
  if (batch < 1) return fail(net->ctx, VARSIM_ERR_INVALID, "batch must be >= 1");
  *bytes = plan(net, batch, training != 0, nullptr).total;
  return VARSIM_OK;
}

varsim_status varsim_net_forward(varsim_net* net, int32_t batch, const float* q_dyn, const float* leak_var,
                                 const float* cond_map, const int32_t* sample_idx, float* dT_out, void* workspace,
                                 size_t ws_bytes, void* stream) {
  if (!net) return VARSIM_ERR_INVALID;
  varsim_ctx* ctx = net->ctx;
  varsim_status st = check_batch(net, batch, q_dyn, workspace, ws_bytes, false);
  if (st != VARSIM_OK) return st;
  if (!dT_out) return fail(ctx, VARSIM_ERR_INVALID, "dT_out is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const NetBufs b = plan(net, batch, false, (char*)workspace);
  st = run_forward(net, batch, q_dyn, leak_var, cond_map, sample_idx, dT_out, b, false, s);
  settle_timing(ctx);
  return st;
}

varsim_status varsim_net_gradient(varsim_net* net, int32_t batch, const float* q_dyn, const float* leak_var,
                                  const float* cond_map, const int32_t* sample_idx, const float* target, float* grad,
                                  float* loss, void* workspace, size_t ws_bytes, void* stream) {
  if (!net) return VARSIM_ERR_INVALID;
  varsim_ctx* ctx = net->ctx;
  varsim_status st = check_batch(net, batch, q_dyn, workspace, ws_bytes, true);
  if (st != VARSIM_OK) return st;
  if (!target || !grad || !loss) return fail(ctx, VARSIM_ERR_INVALID, "target, grad and loss are required");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  const NetBufs b = plan(net, batch, true, (char*)workspace);
  if ((st = run_forward(net, batch, q_dyn, leak_var, cond_map, sample_idx, b.y, b, true, s)) != VARSIM_OK) return st;
  if ((st = run_gradient(net, batch, sample_idx, target, grad, loss, b, s)) != VARSIM_OK) return st;
  settle_timing(ctx);
  return VARSIM_OK;
}

varsim_status varsim_net_adam(varsim_net* net, const float* grad, float lr, float beta1, float beta2, float eps,
                              void* stream) {
  if (!net) return VARSIM_ERR_INVALID;
  varsim_ctx* ctx = net->ctx;
  if (!grad) return fail(ctx, VARSIM_ERR_INVALID, "grad is NULL");
  if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(ctx, VARSIM_ERR_INVALID, "bad Adam hyper-parameters");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  net->adam_t += 1;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, net->adam_t));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, net->adam_t));
  HIP_TRY(timed(ctx, "nn_adam", s,
                [&] { return nn_adam(net->p, net->m, net->v, grad, net->count, lr, beta1, beta2, eps, bc1, bc2, s); }));
  HIP_TRY(refresh_bf16(net, s));
  return VARSIM_OK;
}

varsim_status varsim_nn_conv_workspace(int32_t op, int32_t k, int32_t batch, int32_t h, int32_t w, int32_t cin,
                                       int32_t cout, size_t* bytes) {
  if (!bytes || (k != 1 && k != 3) || batch < 1 || h < 1 || w < 1 || cin < 16 || cout < 16) return VARSIM_ERR_INVALID;
  size_t b = 0;
  if (op == VARSIM_NN_DGRAD) b = up256((size_t)cout * k * k * cin * 2);
  else if (op == VARSIM_NN_WGRAD) b = up256((size_t)nn_wgrad_splits(k, batch, h, w, cin, cout) * cout * k * k * cin * 4);
  else if (op != VARSIM_NN_FWD) return VARSIM_ERR_INVALID;
  *bytes = b;
  return VARSIM_OK;
}

varsim_status varsim_nn_conv(varsim_ctx* ctx, int32_t op, int32_t k, int32_t batch, int32_t h, int32_t w, int32_t cin,
                             int32_t cout, const uint16_t* a, const uint16_t* bw, const float* bias, int32_t relu,
                             void* out, void* workspace, size_t ws_bytes, void* stream) {
  if (!ctx) return VARSIM_ERR_INVALID;
  if (!a || !bw || !out) return fail(ctx, VARSIM_ERR_INVALID, "NULL tensor");
  if ((k != 1 && k != 3) || batch < 1 || h < 1 || w < 1 || cin < 16 || cout < 16 || cin % 16 || cout % 16 ||
      cin > 1024 || cout > 1024)
    return fail(ctx, VARSIM_ERR_UNSUPPORTED, "need k in {1, 3} and channel counts multiples of 16 in [16, 1024]");
  size_t need = 0;
  if (varsim_nn_conv_workspace(op, k, batch, h, w, cin, cout, &need) != VARSIM_OK)
    return fail(ctx, VARSIM_ERR_INVALID, "bad op");
  if (need && (!workspace || ws_bytes < need)) return fail(ctx, VARSIM_ERR_NO_MEMORY, "workspace too small");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  NnConv c{};
  c.B = batch, c.H = h, c.W = w;
  if (op == VARSIM_NN_FWD) {
    c.x = a, c.cx = cin, c.w = bw, c.bias = bias, c.y = out, c.cout = cout;
    HIP_TRY(nn_conv(k, NN_EPI_BF16, relu != 0, c, s));
  } else if (op == VARSIM_NN_DGRAD) {
    uint16_t* wt = (uint16_t*)workspace;
    HIP_TRY(nn_weight_cast_bf16(bw, cout, k * k, cin, cin, nullptr, wt, s));
    c.x = a, c.cx = cout, c.w = wt, c.y = out, c.cout = cin;
    HIP_TRY(nn_conv(k, NN_EPI_F32, false, c, s));
  } else {
    c.x = a, c.cx = cin, c.cout = cout;
    const int ns = nn_wgrad_splits(k, batch, h, w, cin, cout);
    float* part = (float*)workspace;
    HIP_TRY(nn_wgrad(k, c, bw, part, ns, s));
    HIP_TRY(nn_reduce_parts(part, ns, cout, k * k, cin, cin, (float*)out, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return VARSIM_OK;
}

}  // extern "C"
