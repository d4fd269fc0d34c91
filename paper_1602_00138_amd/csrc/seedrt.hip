// Learned-seed network: layer table, forward / backward / Adam schedules and the C ABI
// (rom_seednet_*).  The network (4 levels, 16 -> 64 channels) maps [normalised
// absorption, log diffusion coefficient, source indicator] to a guess of the normalised
// solution; see include/rom.h.  All device memory is caller-owned.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

struct rom_seednet;

namespace rom {
namespace {

constexpr int CIN = 3;        // input fields
constexpr int COUT_MAX = 16;  // output channels: 1 for the guess, up to 16 recycle vectors
constexpr int NL = 8;         // layers

struct Layer {
  const char* name;
  int cin, cout, level;
};
// encoder e0..e3, decoder d2..d0, head (order of the flat parameter vector)
const Layer LAYERS[NL] = {{"e0", CIN, 16, 0}, {"e1", 16, 32, 1}, {"e2", 32, 48, 2},
                          {"e3", 48, 64, 3},  {"d2", 64, 48, 2}, {"d1", 48, 32, 1},
                          {"d0", 32, 16, 0},  {"head", 16, 1, 0}};   // head width: per network

int rows16(int c) { return (c + 15) / 16 * 16; }

struct Arena2 {
  char* base;
  size_t off = 0;
  explicit Arena2(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

}  // namespace
}  // namespace rom

struct rom_seednet {
  int nx, ny, nz, maxb;
  int cout;                  // output channels
  rom::Layer L[rom::NL];     // the layer table with this network's head width
  int64_t nparams;
  // parameters (FP32 master, oracle order), gradients, Adam moments
  float *P, *G, *M, *V;
  int step = 0;
  int64_t woff[rom::NL], boff[rom::NL];
  // per layer GEMM weights, data-gradient weights, GEMM-layout weight-gradient scratch
  void *Wb[rom::NL], *Wt[rom::NL];
  float* dWg[rom::NL];
  int Cpi[rom::NL], Cpo[rom::NL], Kp[rom::NL], rows[rom::NL], Ktp[rom::NL], rowst[rom::NL];
  float *part, *partb;
  double *lpart, *loss;
  // activations (BF16) and their gradients
  void *x, *e0, *p1, *e1, *p2, *e2, *p3, *e3, *d2, *d1, *d0, *y;
  void *ge0, *gp1, *ge1, *gp2, *ge2, *gp3, *ge3, *gu2, *gd2, *gu1, *gd1, *gu0, *gd0, *gy;
  double* hloss = nullptr;   // pinned host copy
};

namespace rom {
namespace {

size_t layout(rom_seednet* net, int nx, int ny, int nz, int maxb, int cout, void* pmem,
              void* wmem, size_t* pbytes, size_t* wbytes) {
  if (nx % 8 || ny % 8 || nz % 8 || nx < 8 || ny < 8 || nz < 8)
    throw Error(ROM_EINVAL, "seed network: grid sizes must be positive multiples of 8");
  if (maxb < 1) throw Error(ROM_EINVAL, "seed network: batch must be >= 1");
  if (cout < 1 || cout > COUT_MAX) throw Error(ROM_EINVAL, "seed network: 1 <= outputs <= 16");
  Layer table[NL];   // this network's layers: the fixed table with its head width
  for (int l = 0; l < NL; ++l) table[l] = LAYERS[l];
  table[NL - 1].cout = cout;
  const int ycp = seed_round8(cout);   // channel slots of the output and its gradient
  int64_t np = 0;
  int64_t woff[NL], boff[NL];
  for (int l = 0; l < NL; ++l) {
    woff[l] = np;
    np += (int64_t)table[l].cout * table[l].cin * 27;
    boff[l] = np;
    np += table[l].cout;
  }
  Arena2 pa(pmem);
  float* P = pa.take<float>(np);
  float* G = pa.take<float>(np);
  float* M = pa.take<float>(np);
  float* V = pa.take<float>(np);
  *pbytes = pa.off + 256;
  Arena2 a(wmem);
  const int64_t n0 = (int64_t)nx * ny * nz * maxb;
  const int64_t nl[4] = {n0, n0 / 8, n0 / 64, n0 / 512};
  size_t part = 0;
  for (int l = 0; l < NL; ++l) {
    const Layer& L = table[l];
    const int cpi = seed_round8(L.cin), cpo = seed_round8(L.cout);
    const int kp = seed_kp(cpi), r = rows16(L.cout), ktp = seed_kp(cpo), rt = rows16(L.cin);
    if (net) {
      net->Cpi[l] = cpi;
      net->Cpo[l] = cpo;
      net->Kp[l] = kp;
      net->rows[l] = r;
      net->Ktp[l] = ktp;
      net->rowst[l] = rt;
    }
    void* wb = a.take<uint16_t>((size_t)r * kp);
    void* wt = a.take<uint16_t>((size_t)rt * ktp);
    float* dw = a.take<float>((size_t)r * kp);
    if (net) {
      net->Wb[l] = wb;
      net->Wt[l] = wt;
      net->dWg[l] = dw;
    }
    const int lev = L.level;
    const int nxl = nx >> lev, nyl = ny >> lev, nzl = nz >> lev;
    part = std::max(part, seed_wgrad_partials(nxl, nyl, nzl, maxb, r, kp));
  }
  float* prt = a.take<float>(part);
  float* prtb = a.take<float>((size_t)(n0 / 2048 + 2) * 64);
  double* lp = a.take<double>(2048);
  double* ls = a.take<double>(8);
  auto act = [&](int lev, int c) { return a.take<uint16_t>((size_t)nl[lev] * c); };
  // the decoder inputs (upsampled e3, d2, d1) are never formed: the layers read them
  void *x = act(0, 8), *e0 = act(0, 16), *p1 = act(1, 16), *e1 = act(1, 32), *p2 = act(2, 32),
       *e2 = act(2, 48), *p3 = act(3, 48), *e3 = act(3, 64), *d2 = act(2, 48), *d1 = act(1, 32),
       *d0 = act(0, 16), *y = act(0, ycp);
  void *ge0 = act(0, 16), *gp1 = act(1, 16), *ge1 = act(1, 32), *gp2 = act(2, 32),
       *ge2 = act(2, 48), *gp3 = act(3, 48), *ge3 = act(3, 64), *gu2 = act(2, 64),
       *gd2 = act(2, 48), *gu1 = act(1, 48), *gd1 = act(1, 32), *gu0 = act(0, 32),
       *gd0 = act(0, 16), *gy = act(0, ycp);
  *wbytes = a.off + 256;
  if (net) {
    net->cout = cout;
    for (int l = 0; l < NL; ++l) net->L[l] = table[l];
    net->nx = nx;
    net->ny = ny;
    net->nz = nz;
    net->maxb = maxb;
    net->nparams = np;
    std::memcpy(net->woff, woff, sizeof(woff));
    std::memcpy(net->boff, boff, sizeof(boff));
    net->P = P;
    net->G = G;
    net->M = M;
    net->V = V;
    net->part = prt;
    net->partb = prtb;
    net->lpart = lp;
    net->loss = ls;
    net->x = x; net->e0 = e0; net->p1 = p1; net->e1 = e1; net->p2 = p2; net->e2 = e2;
    net->p3 = p3; net->e3 = e3; net->d2 = d2; net->d1 = d1; net->d0 = d0; net->y = y;
    net->ge0 = ge0; net->gp1 = gp1; net->ge1 = ge1; net->gp2 = gp2; net->ge2 = ge2;
    net->gp3 = gp3; net->ge3 = ge3; net->gu2 = gu2; net->gd2 = gd2; net->gu1 = gu1;
    net->gd1 = gd1; net->gu0 = gu0; net->gd0 = gd0; net->gy = gy;
  }
  return np;
}

void pack_all(rom_seednet* n, hipStream_t st) {
  for (int l = 0; l < NL; ++l)
    launch_seed_pack_weights(n->P + n->woff[l], n->L[l].cout, n->L[l].cin, n->Cpi[l],
                             n->Kp[l], n->rows[l], n->Wb[l], n->Cpo[l], n->Ktp[l], n->rowst[l],
                             n->Wt[l], st);
}

// forward of one layer: Y = act(conv(X) + b + skip) on the layer's level grid (up: X is
// on the next coarser level and the layer reads its upsampling)
void conv(rom_seednet* n, int l, int b, const void* X, const void* skip, bool relu, void* Y,
          hipStream_t st, bool up = false) {
  const int lev = n->L[l].level;
  launch_seed_conv(n->nx >> lev, n->ny >> lev, n->nz >> lev, b, X, n->Cpi[l], n->Wb[l], n->Kp[l],
                   n->L[l].cout, n->rows[l], n->P + n->boff[l], skip, relu ? 1 : 0, Y,
                   n->Cpo[l], st, up ? 1 : 0);
}

// data gradient of layer l: dX = conv(dZ; flipped, transposed weights)
void conv_dx(rom_seednet* n, int l, int b, const void* dZ, void* dX, hipStream_t st) {
  const int lev = n->L[l].level;
  launch_seed_conv(n->nx >> lev, n->ny >> lev, n->nz >> lev, b, dZ, n->Cpo[l], n->Wt[l],
                   n->Ktp[l], n->L[l].cin, n->rowst[l], nullptr, nullptr, 0, dX, n->Cpi[l], st);
}

// weight and bias gradients of layer l (added into G; up as for the forward)
void conv_dw(rom_seednet* n, int l, int b, const void* X, const void* dZ, hipStream_t st,
             bool up = false) {
  const int lev = n->L[l].level;
  launch_seed_wgrad(n->nx >> lev, n->ny >> lev, n->nz >> lev, b, X, n->Cpi[l], dZ, n->Cpo[l],
                    n->L[l].cout, n->rows[l], n->Kp[l], n->part, n->dWg[l], n->partb,
                    n->G + n->boff[l], st, up ? 1 : 0);
  launch_seed_unpack_wgrad(n->dWg[l], n->Kp[l], n->L[l].cout, n->L[l].cin, n->Cpi[l],
                           n->G + n->woff[l], st);
}

int64_t nvox(const rom_seednet* n, int lev, int b) {
  return (int64_t)(n->nx >> lev) * (n->ny >> lev) * (n->nz >> lev) * b;
}

void forward(rom_seednet* n, const float* in, int b, hipStream_t st) {
  const int nx = n->nx, ny = n->ny, nz = n->nz;
  launch_seed_pack_input((int64_t)nx * ny * nz, b, CIN, in, n->x, 8, st);
  conv(n, 0, b, n->x, nullptr, true, n->e0, st);
  launch_seed_pool(nx, ny, nz, b, n->e0, n->p1, 16, st);
  conv(n, 1, b, n->p1, nullptr, true, n->e1, st);
  launch_seed_pool(nx / 2, ny / 2, nz / 2, b, n->e1, n->p2, 32, st);
  conv(n, 2, b, n->p2, nullptr, true, n->e2, st);
  launch_seed_pool(nx / 4, ny / 4, nz / 4, b, n->e2, n->p3, 48, st);
  conv(n, 3, b, n->p3, nullptr, true, n->e3, st);
  // the decoder layers read the upsampling of the coarser level directly
  conv(n, 4, b, n->e3, n->e2, true, n->d2, st, true);
  conv(n, 5, b, n->d2, n->e1, true, n->d1, st, true);
  conv(n, 6, b, n->d1, n->e0, true, n->d0, st, true);
  conv(n, 7, b, n->d0, nullptr, false, n->y, st);
}

// gradients of every layer added into G (the caller zeros G) from the output gradient in gy
void backward_layers(rom_seednet* n, int b, hipStream_t st) {
  const int nx = n->nx, ny = n->ny, nz = n->nz;
  // head (no activation)
  conv_dw(n, 7, b, n->d0, n->gy, st);
  conv_dx(n, 7, b, n->gy, n->gd0, st);
  // d0 = relu(conv(u0) + e0)
  launch_seed_relu_bwd(nvox(n, 0, b) * 16, n->gd0, n->d0, st);
  conv_dw(n, 6, b, n->d1, n->gd0, st, true);
  conv_dx(n, 6, b, n->gd0, n->gu0, st);
  ROM_HIP(hipMemcpyAsync(n->ge0, n->gd0, nvox(n, 0, b) * 16 * 2, hipMemcpyDeviceToDevice, st));
  launch_seed_up_bwd(nx, ny, nz, b, n->gu0, n->gd1, 32, st);
  // d1
  launch_seed_relu_bwd(nvox(n, 1, b) * 32, n->gd1, n->d1, st);
  conv_dw(n, 5, b, n->d2, n->gd1, st, true);
  conv_dx(n, 5, b, n->gd1, n->gu1, st);
  ROM_HIP(hipMemcpyAsync(n->ge1, n->gd1, nvox(n, 1, b) * 32 * 2, hipMemcpyDeviceToDevice, st));
  launch_seed_up_bwd(nx / 2, ny / 2, nz / 2, b, n->gu1, n->gd2, 48, st);
  // d2
  launch_seed_relu_bwd(nvox(n, 2, b) * 48, n->gd2, n->d2, st);
  conv_dw(n, 4, b, n->e3, n->gd2, st, true);
  conv_dx(n, 4, b, n->gd2, n->gu2, st);
  ROM_HIP(hipMemcpyAsync(n->ge2, n->gd2, nvox(n, 2, b) * 48 * 2, hipMemcpyDeviceToDevice, st));
  launch_seed_up_bwd(nx / 4, ny / 4, nz / 4, b, n->gu2, n->ge3, 64, st);
  // e3
  launch_seed_relu_bwd(nvox(n, 3, b) * 64, n->ge3, n->e3, st);
  conv_dw(n, 3, b, n->p3, n->ge3, st);
  conv_dx(n, 3, b, n->ge3, n->gp3, st);
  launch_seed_pool_bwd(nx / 4, ny / 4, nz / 4, b, n->gp3, n->ge2, 48, 1, st);
  // e2
  launch_seed_relu_bwd(nvox(n, 2, b) * 48, n->ge2, n->e2, st);
  conv_dw(n, 2, b, n->p2, n->ge2, st);
  conv_dx(n, 2, b, n->ge2, n->gp2, st);
  launch_seed_pool_bwd(nx / 2, ny / 2, nz / 2, b, n->gp2, n->ge1, 32, 1, st);
  // e1
  launch_seed_relu_bwd(nvox(n, 1, b) * 32, n->ge1, n->e1, st);
  conv_dw(n, 1, b, n->p1, n->ge1, st);
  conv_dx(n, 1, b, n->ge1, n->gp1, st);
  launch_seed_pool_bwd(nx, ny, nz, b, n->gp1, n->ge0, 16, 1, st);
  // e0
  launch_seed_relu_bwd(nvox(n, 0, b) * 16, n->ge0, n->e0, st);
  conv_dw(n, 0, b, n->x, n->ge0, st);
}

// MSE loss of the single output channel (into n->loss[0]) and gradients added into G
void backward(rom_seednet* n, const float* target, int b, hipStream_t st) {
  launch_seed_mse(nvox(n, 0, b), n->y, n->Cpo[NL - 1], target, n->gy, n->lpart, n->loss, st);
  backward_layers(n, b, st);
}

void adam_step(rom_seednet* n, float lr, hipStream_t st) {
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
  launch_seed_adam(n->nparams, n->P, n->G, n->M, n->V, lr, b1, b2, c1, c2, 1e-8f, st);
  pack_all(n, st);
}

void check_batch(const rom_seednet* n, int b) {
  if (!n) throw Error(ROM_EINVAL, "null network");
  if (b < 1 || b > n->maxb) throw Error(ROM_EINVAL, "batch out of range");
}

void check_single(const rom_seednet* n) {
  if (n->cout != 1) throw Error(ROM_EINVAL, "the MSE loss needs a network with one output");
}

}  // namespace
}  // namespace rom

using rom::Error;

extern "C" {

rom_status rom_seednet_bytes(int nx, int ny, int nz, int batch, int outputs, int64_t* nparams,
                             size_t* param_bytes, size_t* work_bytes) {
  try {
    if (!nparams || !param_bytes || !work_bytes) throw Error(ROM_EINVAL, "null argument");
    *nparams = (int64_t)rom::layout(nullptr, nx, ny, nz, batch, outputs, nullptr, nullptr,
                                    param_bytes, work_bytes);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_create(int nx, int ny, int nz, int batch, int outputs, const float* params,
                              void* param_mem, size_t param_bytes, void* work_mem,
                              size_t work_bytes, rom_seednet** net, void* stream) {
  try {
    if (!params || !param_mem || !work_mem || !net) throw Error(ROM_EINVAL, "null argument");
    size_t pb = 0, wb = 0;
    rom::layout(nullptr, nx, ny, nz, batch, outputs, nullptr, nullptr, &pb, &wb);
    if (param_bytes < pb || work_bytes < wb) throw Error(ROM_ECAPACITY, "buffers too small");
    if ((uintptr_t)param_mem % 256 || (uintptr_t)work_mem % 256)
      throw Error(ROM_EINVAL, "buffers must be 256-byte aligned");
    rom_seednet* n = new rom_seednet;
    rom::layout(n, nx, ny, nz, batch, outputs, param_mem, work_mem, &pb, &wb);
    hipStream_t st = (hipStream_t)stream;
    try {
      ROM_HIP(hipHostMalloc((void**)&n->hloss, sizeof(double), hipHostMallocDefault));
      ROM_HIP(hipMemcpyAsync(n->P, params, n->nparams * sizeof(float), hipMemcpyHostToDevice, st));
      ROM_HIP(hipMemsetAsync(n->M, 0, n->nparams * sizeof(float), st));
      ROM_HIP(hipMemsetAsync(n->V, 0, n->nparams * sizeof(float), st));
      rom::pack_all(n, st);
      ROM_HIP(hipStreamSynchronize(st));
    } catch (...) {
      delete n;
      throw;
    }
    *net = n;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_forward(rom_seednet* net, const float* in, float* out, int batch,
                               void* stream) {
  try {
    rom::check_batch(net, batch);
    if (!in || !out) throw Error(ROM_EINVAL, "null input or output");
    hipStream_t st = (hipStream_t)stream;
    rom::forward(net, in, batch, st);
    rom::launch_seed_unpack_output(rom::nvox(net, 0, 1), batch, net->cout, net->y,
                                   net->Cpo[rom::NL - 1], out, st);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_gradients(rom_seednet* net, const float* in, const float* target,
                                 int batch, float* grads, double* loss, void* stream) {
  try {
    rom::check_batch(net, batch);
    if (!in || !target) throw Error(ROM_EINVAL, "null input or target");
    rom::check_single(net);
    hipStream_t st = (hipStream_t)stream;
    ROM_HIP(hipMemsetAsync(net->G, 0, net->nparams * sizeof(float), st));
    rom::forward(net, in, batch, st);
    rom::backward(net, target, batch, st);
    if (grads)
      ROM_HIP(hipMemcpyAsync(grads, net->G, net->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipMemcpyAsync(net->hloss, net->loss, sizeof(double), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    if (loss) *loss = *net->hloss;
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_train_step(rom_seednet* net, const float* in, const float* target,
                                  int batch, float lr, double* loss, void* stream) {
  try {
    rom::check_batch(net, batch);
    if (!in || !target) throw Error(ROM_EINVAL, "null input or target");
    if (!(lr > 0.f)) throw Error(ROM_EINVAL, "learning rate must be > 0");
    rom::check_single(net);
    hipStream_t st = (hipStream_t)stream;
    ROM_HIP(hipMemsetAsync(net->G, 0, net->nparams * sizeof(float), st));
    rom::forward(net, in, batch, st);
    rom::backward(net, target, batch, st);
    rom::adam_step(net, lr, st);
    if (loss) {
      ROM_HIP(hipMemcpyAsync(net->hloss, net->loss, sizeof(double), hipMemcpyDeviceToHost, st));
      ROM_HIP(hipStreamSynchronize(st));
      *loss = *net->hloss;
    }
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_backward(rom_seednet* net, const float* in, const float* dy, int batch,
                                float* grads, void* stream) {
  try {
    rom::check_batch(net, batch);
    if (!in || !dy) throw Error(ROM_EINVAL, "null input or output gradient");
    hipStream_t st = (hipStream_t)stream;
    ROM_HIP(hipMemsetAsync(net->G, 0, net->nparams * sizeof(float), st));
    rom::forward(net, in, batch, st);
    rom::launch_seed_pack_input(rom::nvox(net, 0, 1), batch, net->cout, dy, net->gy,
                                net->Cpo[rom::NL - 1], st);
    rom::backward_layers(net, batch, st);
    if (grads) {
      ROM_HIP(hipMemcpyAsync(grads, net->G, net->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
      ROM_HIP(hipStreamSynchronize(st));
    }
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_adam(rom_seednet* net, float lr, void* stream) {
  try {
    if (!net) throw Error(ROM_EINVAL, "null network");
    if (!(lr > 0.f)) throw Error(ROM_EINVAL, "learning rate must be > 0");
    rom::adam_step(net, lr, (hipStream_t)stream);
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

rom_status rom_seednet_params(const rom_seednet* net, float* params, void* stream) {
  try {
    if (!net || !params) throw Error(ROM_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    ROM_HIP(hipMemcpyAsync(params, net->P, net->nparams * sizeof(float), hipMemcpyDeviceToHost, st));
    ROM_HIP(hipStreamSynchronize(st));
    return ROM_OK;
  } catch (const Error& e) {
    return rom::report(e);
  }
}

void rom_seednet_destroy(rom_seednet* net) {
  if (!net) return;
  if (net->hloss) (void)hipHostFree(net->hloss);
  delete net;
}

}  // extern "C"
