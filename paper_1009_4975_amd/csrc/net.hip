// Learned warm start: a small fully convolutional network on a regular grid
// (FP32), trained and evaluated on the GPU by the kernels below, and the
// transfers between the finite-element mesh and that grid.
//
// Network: n_layers 3x3x3 convolutions (stride 1, zero padding 1) with ReLU
// between layers and none after the last.  Activations (B, C, Z, Y, X),
// weights (Cout, Cin, 3, 3, 3).  The grids are small (tens of thousands of
// cells), so the convolutions are direct: one thread per output value for the
// forward and data-gradient passes, one workgroup per weight for the
// weight-gradient reduction (deterministic tree sums).
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"

struct amrto_net {
  int device = 0;
  hipStream_t stream = nullptr;
  int L = 0;
  int skip = -1;           // output += input channels [skip, skip + C_L) (-1: none)
  std::vector<int> ch;     // L + 1 channel counts
  int gx = 0, gy = 0, gz = 0, max_batch = 0, batch = 0;
  std::vector<long> woff;  // parameter offsets: w_l at woff[l], b_l after it
  long n_params = 0;
  float* d_params = nullptr;
  float* d_grads = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  std::vector<float*> acts;  // acts[0] = input copy, acts[l + 1] = output of layer l (post-ReLU except last)
  float* d_tmp0 = nullptr;   // gradient buffers (max activation size)
  float* d_tmp1 = nullptr;
  double* d_red = nullptr;
  std::string err;
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

namespace amrto {

__device__ __forceinline__ bool in_grid(int z, int y, int x, int Z, int Y, int X) {
  return z >= 0 && z < Z && y >= 0 && y < Y && x >= 0 && x < X;
}

// out[n, o, p] = b[o] + sum_{i, d} w[o, i, d] in[n, i, p + d - 1]; optional ReLU
__global__ __launch_bounds__(256) void k_conv_fwd(const float* __restrict__ in, const float* __restrict__ w,
                                                  const float* __restrict__ b, float* __restrict__ out, int B,
                                                  int Ci, int Co, int Z, int Y, int X, int relu) {
  const long V = (long)Z * Y * X;
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)B * Co * V) return;
  const long p = idx % V;
  const int o = (int)((idx / V) % Co), n = (int)(idx / (V * Co));
  const int x = p % X, y = (p / X) % Y, z = (int)(p / ((long)X * Y));
  float acc = b[o];
  for (int i = 0; i < Ci; ++i) {
    const float* src = in + ((long)n * Ci + i) * V;
    const float* wk = w + ((long)o * Ci + i) * 27;
#pragma unroll
    for (int d = 0; d < 27; ++d) {
      const int zz = z + d / 9 - 1, yy = y + (d / 3) % 3 - 1, xx = x + d % 3 - 1;
      if (in_grid(zz, yy, xx, Z, Y, X)) acc = fmaf(wk[d], src[((long)zz * Y + yy) * X + xx], acc);
    }
  }
  out[idx] = relu ? fmaxf(acc, 0.f) : acc;
}

// din[n, i, p] = sum_{o, d} w[o, i, d] g[n, o, p - d + 1], g masked by ReLU of `post` (if given)
__global__ __launch_bounds__(256) void k_conv_bwd_data(const float* __restrict__ g, const float* __restrict__ post,
                                                       const float* __restrict__ w, float* __restrict__ din, int B,
                                                       int Ci, int Co, int Z, int Y, int X) {
  const long V = (long)Z * Y * X;
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)B * Ci * V) return;
  const long p = idx % V;
  const int i = (int)((idx / V) % Ci), n = (int)(idx / (V * Ci));
  const int x = p % X, y = (p / X) % Y, z = (int)(p / ((long)X * Y));
  float acc = 0.f;
  for (int o = 0; o < Co; ++o) {
    const float* go = g + ((long)n * Co + o) * V;
    const float* po = post ? post + ((long)n * Co + o) * V : nullptr;
    const float* wk = w + ((long)o * Ci + i) * 27;
#pragma unroll
    for (int d = 0; d < 27; ++d) {
      const int zz = z - (d / 9 - 1), yy = y - ((d / 3) % 3 - 1), xx = x - (d % 3 - 1);
      if (in_grid(zz, yy, xx, Z, Y, X)) {
        const long q = ((long)zz * Y + yy) * X + xx;
        if (!po || po[q] > 0.f) acc = fmaf(wk[d], go[q], acc);
      }
    }
  }
  din[idx] = acc;
}

// dw[o, i, d] = sum_{n, p} g[n, o, p] in[n, i, p + d - 1]; db[o] = sum g (one block per weight)
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const float* __restrict__ g, const float* __restrict__ post,
                                                         const float* __restrict__ in, float* __restrict__ dw,
                                                         float* __restrict__ db, int B, int Ci, int Co, int Z,
                                                         int Y, int X) {
  __shared__ double sh[8];
  const int wid = blockIdx.x;  // o * (Ci * 27 + 1) + (i * 27 + d) or the bias slot
  const int per = Ci * 27 + 1;
  const int o = wid / per, r = wid % per;
  const bool bias = r == Ci * 27;
  const int i = bias ? 0 : r / 27, d = bias ? 0 : r % 27;
  const int oz = d / 9 - 1, oy = (d / 3) % 3 - 1, ox = d % 3 - 1;
  const long V = (long)Z * Y * X;
  double acc = 0.0;
  for (long t = threadIdx.x; t < (long)B * V; t += blockDim.x) {
    const int n = (int)(t / V);
    const long p = t % V;
    const long gi = ((long)n * Co + o) * V + p;
    float gv = g[gi];
    if (post && !(post[gi] > 0.f)) gv = 0.f;
    if (bias) { acc += gv; continue; }
    const int x = p % X, y = (p / X) % Y, z = (int)(p / ((long)X * Y));
    const int zz = z + oz, yy = y + oy, xx = x + ox;
    if (in_grid(zz, yy, xx, Z, Y, X)) acc += (double)gv * in[((long)n * Ci + i) * V + ((long)zz * Y + yy) * X + xx];
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (bias) db[o] = (float)acc;
    else dw[((long)o * Ci + i) * 27 + d] = (float)acc;
  }
}

// masked MSE: partial sums of mask (p - t)^2 and of mask; dpred = 2 mask (p - t) / sum(mask)
__global__ __launch_bounds__(256) void k_mse_part(const float* __restrict__ p, const float* __restrict__ t,
                                                  const uint8_t* __restrict__ m, long n, double* __restrict__ part) {
  __shared__ double sh[8];
  double s = 0.0, c = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (!m || m[i]) {
      const double d = (double)p[i] - (double)t[i];
      s += d * d;
      c += 1.0;
    }
  s = block_sum(s, sh);
  c = block_sum(c, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[RED_BLOCKS + blockIdx.x] = c;
  }
}

__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ p, const float* __restrict__ t,
                                                  const uint8_t* __restrict__ m, long n,
                                                  const double* __restrict__ part, float* __restrict__ dp,
                                                  double* __restrict__ out) {
  __shared__ double sh[8];
  const double s = sum_partials(part, RED_BLOCKS, sh);
  const double c = sum_partials(part + RED_BLOCKS, RED_BLOCKS, sh);
  const double inv = c > 0 ? 1.0 / c : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = s * inv;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dp[i] = (!m || m[i]) ? (float)(2.0 * ((double)p[i] - (double)t[i]) * inv) : 0.f;
}

// out[n, oo + c, p] += in[n, io + c, p] for c < C (residual connection around
// the stack; out has Co channels, in has Ci)
__global__ __launch_bounds__(256) void k_add_skip(float* __restrict__ out, int Co, int oo, const float* __restrict__ in,
                                                  int Ci, int io, int C, int B, long V) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)B * C * V) return;
  const long p = idx % V;
  const int c = (int)((idx / V) % C), n = (int)(idx / (V * C));
  out[((long)n * Co + oo + c) * V + p] += in[((long)n * Ci + io + c) * V + p];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ mesh <-> grid
// rho_grid[g] = sum over the elements overlapping the dual cell of grid node g
// of rho_e times the overlapped fraction of that cell (fixed order: deterministic)
__global__ __launch_bounds__(256) void k_grid_density(const double* __restrict__ rho, const int32_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ elem, const double* __restrict__ w,
                                                      int n_gn, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_gn) return;
  double s = 0.0;
  for (int k = ptr[c]; k < ptr[c + 1]; ++k) s += w[k] * rho[elem[k]];
  out[c] = (float)s;
}

// u_grid[c][g] = scale sum_a w[8 g + a] (u - u_ref)[3 node[8 g + a] + c]
__global__ __launch_bounds__(256) void k_grid_sample(const double* __restrict__ u, const double* __restrict__ uref,
                                                     const int32_t* __restrict__ node, const float* __restrict__ w,
                                                     long n_gn, double scale, float* __restrict__ out) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= 3 * n_gn) return;
  const int c = (int)(i / n_gn);
  const long g = i % n_gn;
  double v = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const long d = 3L * node[8 * g + a] + c;
    v += (double)w[8 * g + a] * (uref ? u[d] - uref[d] : u[d]);
  }
  out[i] = (float)(scale * v);
}

// u[3 n + c] = scale x trilinear interpolation of u_grid[c] at the node's lattice position
__global__ __launch_bounds__(256) void k_grid_interp(const float* __restrict__ ug, const int32_t* __restrict__ xyz,
                                                     int n_nodes, int cell, int gx, int gy, int gz, double scale,
                                                     double* __restrict__ u, int sx, int sy) {
  const int nd = blockIdx.x * blockDim.x + threadIdx.x;
  if (nd >= n_nodes) return;
  int px, py, pz;
  if (xyz) {
    px = xyz[3L * nd]; py = xyz[3L * nd + 1]; pz = xyz[3L * nd + 2];
  } else {
    px = nd % sx; py = (nd / sx) % sy; pz = nd / (sx * sy);
  }
  const int ix = min(px / cell, gx - 1), iy = min(py / cell, gy - 1), iz = min(pz / cell, gz - 1);
  const double tx = (double)(px - ix * cell) / cell, ty = (double)(py - iy * cell) / cell,
               tz = (double)(pz - iz * cell) / cell;
  const long NX = gx + 1, NY = gy + 1, NN = NX * NY * (gz + 1);
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
      const double w = (ax ? tx : 1.0 - tx) * (ay ? ty : 1.0 - ty) * (az ? tz : 1.0 - tz);
      v += w * ug[c * NN + ((iz + az) * NY + iy + ay) * NX + ix + ax];
    }
    u[3L * nd + c] = scale * v;
  }
}

static uint64_t splitmix64(uint64_t x) {
  // SplitMix64 (Steele, Lea, Flood 2014) output function of state x
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

}  // namespace amrto

using namespace amrto;

#define NET_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return net->fail(AMRTO_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

extern "C" {

int amrto_net_create(amrto_net** out, int device, void* stream, int32_t n_layers, const int32_t* channels,
                     int32_t skip_from, int32_t gx, int32_t gy, int32_t gz, int32_t max_batch, uint64_t seed) {
  if (!out || !channels || n_layers < 1 || n_layers > 16 || gx < 1 || gy < 1 || gz < 1 || max_batch < 1)
    return AMRTO_EINVAL;
  if (skip_from >= 0 && skip_from + channels[n_layers] > channels[0]) return AMRTO_EINVAL;
  for (int l = 0; l <= n_layers; ++l)
    if (channels[l] < 1 || channels[l] > 256) return AMRTO_EINVAL;
  amrto_net* net = new (std::nothrow) amrto_net();
  if (!net) return AMRTO_ENOMEM;
  *out = nullptr;
  net->device = device;
  net->stream = (hipStream_t)stream;
  net->L = n_layers;
  net->skip = skip_from < 0 ? -1 : skip_from;
  net->ch.assign(channels, channels + n_layers + 1);
  net->gx = gx; net->gy = gy; net->gz = gz; net->max_batch = max_batch;
  long off = 0;
  for (int l = 0; l < n_layers; ++l) {
    net->woff.push_back(off);
    off += (long)channels[l + 1] * channels[l] * 27 + channels[l + 1];
  }
  net->n_params = off;
  if (hipSetDevice(device) != hipSuccess) { delete net; return AMRTO_EHIP; }
  const long V = (long)gx * gy * gz;
  int cmax = 0;
  for (int c : net->ch) cmax = std::max(cmax, c);
  bool ok = hipMalloc((void**)&net->d_params, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_grads, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_m, off * 4) == hipSuccess && hipMalloc((void**)&net->d_v, off * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_tmp0, (long)max_batch * cmax * V * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_tmp1, (long)max_batch * cmax * V * 4) == hipSuccess &&
            hipMalloc((void**)&net->d_red, 4 * RED_BLOCKS * sizeof(double)) == hipSuccess;
  for (int l = 0; l <= n_layers && ok; ++l) {
    float* p = nullptr;
    ok = hipMalloc((void**)&p, (long)max_batch * channels[l] * V * 4) == hipSuccess;
    net->acts.push_back(p);
  }
  if (!ok) { amrto_net_destroy(net); return AMRTO_ENOMEM; }
  // He-normal weights from a counter-based generator (SplitMix64 + Box-Muller), zero biases
  std::vector<float> h(off, 0.f);
  for (int l = 0; l < n_layers; ++l) {
    const long nw = (long)channels[l + 1] * channels[l] * 27;
    const double sd = std::sqrt(2.0 / (27.0 * channels[l]));
    for (long k = 0; k < nw; ++k) {
      const uint64_t a = splitmix64(seed ^ (uint64_t)(net->woff[l] + k) * 2ULL);
      const uint64_t b = splitmix64(seed ^ ((uint64_t)(net->woff[l] + k) * 2ULL + 1ULL));
      const double u1 = ((a >> 11) + 1.0) / 9007199254740993.0, u2 = (b >> 11) / 9007199254740992.0;
      h[net->woff[l] + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  if (hipMemcpy(net->d_params, h.data(), off * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(net->d_m, 0, off * 4) != hipSuccess || hipMemset(net->d_v, 0, off * 4) != hipSuccess) {
    amrto_net_destroy(net);
    return AMRTO_EHIP;
  }
  *out = net;
  return AMRTO_OK;
}

int amrto_net_destroy(amrto_net* net) {
  if (!net) return AMRTO_OK;
  (void)hipSetDevice(net->device);
  (void)hipDeviceSynchronize();
  for (float* p : {net->d_params, net->d_grads, net->d_m, net->d_v, net->d_tmp0, net->d_tmp1})
    if (p) (void)hipFree(p);
  for (float* p : net->acts)
    if (p) (void)hipFree(p);
  if (net->d_red) (void)hipFree(net->d_red);
  delete net;
  return AMRTO_OK;
}

const char* amrto_net_last_error(const amrto_net* net) { return net ? net->err.c_str() : "null network"; }

int amrto_net_n_params(const amrto_net* net, int64_t* n) {
  if (!net || !n) return AMRTO_EINVAL;
  *n = net->n_params;
  return AMRTO_OK;
}

int amrto_net_get_params(const amrto_net* net, float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(host, net->d_params, net->n_params * 4, hipMemcpyDeviceToHost) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_set_params(amrto_net* net, const float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(net->d_params, host, net->n_params * 4, hipMemcpyHostToDevice) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_get_grads(const amrto_net* net, float* host) {
  if (!net || !host) return AMRTO_EINVAL;
  return hipMemcpy(host, net->d_grads, net->n_params * 4, hipMemcpyDeviceToHost) == hipSuccess ? AMRTO_OK : AMRTO_EHIP;
}

int amrto_net_get_adam(const amrto_net* net, float* m_host, float* v_host) {
  if (!net || !m_host || !v_host) return AMRTO_EINVAL;
  const size_t bytes = net->n_params * 4;
  return hipMemcpy(m_host, net->d_m, bytes, hipMemcpyDeviceToHost) == hipSuccess &&
                 hipMemcpy(v_host, net->d_v, bytes, hipMemcpyDeviceToHost) == hipSuccess
             ? AMRTO_OK
             : AMRTO_EHIP;
}

int amrto_net_set_adam(amrto_net* net, const float* m_host, const float* v_host) {
  if (!net || !m_host || !v_host) return AMRTO_EINVAL;
  for (int64_t i = 0; i < net->n_params; ++i)
    if (!std::isfinite(m_host[i]) || !std::isfinite(v_host[i]) || v_host[i] < 0.f)
      return net->fail(AMRTO_EINVAL, "amrto_net_set_adam: moments must be finite, second moments >= 0");
  const size_t bytes = net->n_params * 4;
  return hipMemcpy(net->d_m, m_host, bytes, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(net->d_v, v_host, bytes, hipMemcpyHostToDevice) == hipSuccess
             ? AMRTO_OK
             : AMRTO_EHIP;
}

int amrto_net_forward(amrto_net* net, const float* in, int32_t batch, float* out) {
  if (!net || !in || batch < 1 || batch > net->max_batch) return net ? net->fail(AMRTO_EINVAL, "amrto_net_forward: bad arguments") : AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const long V = (long)net->gx * net->gy * net->gz;
  net->batch = batch;
  NET_HIP(hipMemcpyAsync(net->acts[0], in, (long)batch * net->ch[0] * V * 4, hipMemcpyDeviceToDevice, net->stream));
  for (int l = 0; l < net->L; ++l) {
    const long n = (long)batch * net->ch[l + 1] * V;
    const float* w = net->d_params + net->woff[l];
    const float* b = w + (long)net->ch[l + 1] * net->ch[l] * 27;
    hipLaunchKernelGGL(k_conv_fwd, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->acts[l], w, b,
                       net->acts[l + 1], batch, net->ch[l], net->ch[l + 1], net->gz, net->gy, net->gx,
                       l + 1 < net->L ? 1 : 0);
  }
  if (net->skip >= 0) {
    const long n = (long)batch * net->ch[net->L] * V;
    hipLaunchKernelGGL(k_add_skip, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->acts[net->L],
                       net->ch[net->L], 0, net->acts[0], net->ch[0], net->skip, net->ch[net->L], batch, V);
  }
  if (out)
    NET_HIP(hipMemcpyAsync(out, net->acts[net->L], (long)batch * net->ch[net->L] * V * 4, hipMemcpyDeviceToDevice,
                           net->stream));
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_net_backward(amrto_net* net, const float* dout, float* din) {
  if (!net || !dout || net->batch < 1) return net ? net->fail(AMRTO_ESTATE, "amrto_net_backward: no forward pass") : AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const int B = net->batch;
  const long V = (long)net->gx * net->gy * net->gz;
  const float* g = dout;
  float* bufs[2] = {net->d_tmp0, net->d_tmp1};
  for (int l = net->L - 1; l >= 0; --l) {
    const int Ci = net->ch[l], Co = net->ch[l + 1];
    const float* post = l + 1 < net->L ? net->acts[l + 1] : nullptr;  // ReLU mask of this layer's output
    float* w = net->d_params + net->woff[l];
    float* dw = net->d_grads + net->woff[l];
    hipLaunchKernelGGL(k_conv_bwd_weight, dim3(Co * (Ci * 27 + 1)), dim3(256), 0, net->stream, g, post,
                       net->acts[l], dw, dw + (long)Co * Ci * 27, B, Ci, Co, net->gz, net->gy, net->gx);
    if (l > 0 || din) {
      float* dst = l > 0 ? bufs[l & 1] : din;
      const long n = (long)B * Ci * V;
      hipLaunchKernelGGL(k_conv_bwd_data, dim3((n + 255) / 256), dim3(256), 0, net->stream, g, post, w, dst, B, Ci,
                         Co, net->gz, net->gy, net->gx);
      g = dst;
    }
  }
  if (din && net->skip >= 0) {
    const long n = (long)B * net->ch[net->L] * V;
    hipLaunchKernelGGL(k_add_skip, dim3((n + 255) / 256), dim3(256), 0, net->stream, din, net->ch[0], net->skip, dout,
                       net->ch[net->L], 0, net->ch[net->L], B, V);
  }
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_net_mse(amrto_net* net, const float* pred, const float* tgt, const uint8_t* mask, int64_t n, float* dpred,
                  double* loss_host) {
  if (!net || !pred || !tgt || !dpred || n < 1) return AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  hipLaunchKernelGGL(k_mse_part, dim3(RED_BLOCKS), dim3(256), 0, net->stream, pred, tgt, mask, (long)n, net->d_red);
  hipLaunchKernelGGL(k_mse_grad, dim3(RED_BLOCKS), dim3(256), 0, net->stream, pred, tgt, mask, (long)n, net->d_red,
                     dpred, net->d_red + 2 * RED_BLOCKS);
  NET_HIP(hipGetLastError());
  if (loss_host) {
    NET_HIP(hipMemcpyAsync(loss_host, net->d_red + 2 * RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, net->stream));
    NET_HIP(hipStreamSynchronize(net->stream));
  }
  return AMRTO_OK;
}

int amrto_net_adam(amrto_net* net, float lr, float b1, float b2, float eps, int32_t t) {
  if (!net || t < 1) return AMRTO_EINVAL;
  NET_HIP(hipSetDevice(net->device));
  const long n = net->n_params;
  const float c1 = 1.f - std::pow(b1, (float)t), c2 = 1.f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->d_params, net->d_grads, net->d_m,
                     net->d_v, n, lr, b1, b2, eps, c1, c2);
  NET_HIP(hipGetLastError());
  return AMRTO_OK;
}

// ------------------------------------------------------------------ mesh <-> grid
// Host tables of the transfers for grid cells of edge `cell` lattice units:
// the elements overlapping each cell with their overlap fractions, and for
// each grid node the element containing it with the trilinear weights of that
// element's vertices (exact at mesh nodes; at a hanging node it equals the
// constrained value of Eq. (6)).
static int grid_maps(amrto_ctx* ctx, int cell) {
  if (ctx->grid_cell == cell) return AMRTO_OK;
  if (cell < 1 || ctx->nx % cell || ctx->ny % cell || ctx->nz % cell)
    return ctx->fail(AMRTO_EINVAL, "grid: cell must divide the domain");
  const int gx = ctx->nx / cell, gy = ctx->ny / cell, gz = ctx->nz / cell;
  const long NX = gx + 1, NY = gy + 1, n_gn = NX * NY * (gz + 1);
  const int ne = ctx->n_elems;
  std::vector<int32_t> celem, fill;
  std::vector<double> cw;
  auto elem_geom = [&](int e, int* p, int* vert) -> int {
    if (ctx->uniform) {
      const int ex = e % ctx->nx, ey = (e / ctx->nx) % ctx->ny, ez = e / (ctx->nx * ctx->ny);
      p[0] = ex; p[1] = ey; p[2] = ez;
      for (int a = 0; a < 8; ++a)
        vert[a] = (ex + (a & 1)) + (ctx->nx + 1) * ((ey + ((a >> 1) & 1)) + (ctx->ny + 1) * (ez + (a >> 2)));
      return 1;
    }
    for (int a = 0; a < 8; ++a) vert[a] = ctx->h_elem_nodes[8L * e + a];
    const int* q = &ctx->h_node_xyz[3L * vert[0]];
    p[0] = q[0]; p[1] = q[1]; p[2] = q[2];
    return 1 << (ctx->max_level - ctx->h_level[e]);
  };
  // grid node -> elements overlapping its dual cell (the box of edge `cell`
  // centred at the node, clipped to the domain); doubled coordinates keep the
  // half-cell offsets integral.  Counting pass, then fill in element order.
  const int dims[3] = {ctx->nx, ctx->ny, ctx->nz};
  const int gdim[3] = {gx, gy, gz};
  int p[3], vert[8];
  auto node_range = [&](int ax, int lo, int h, int& n0, int& n1) {
    n0 = std::max(0, (2 * lo - cell) / (2 * cell) - 1);
    n1 = std::min(gdim[ax], (2 * (lo + h) + cell) / (2 * cell) + 1);
  };
  auto overlap2 = [&](int ax, int i, int lo, int h) -> long {
    const long b0 = std::max(0L, 2L * i * cell - cell), b1 = std::min(2L * dims[ax], 2L * i * cell + cell);
    return std::max(0L, std::min(b1, 2L * (lo + h)) - std::max(b0, 2L * lo));
  };
  auto box2 = [&](int ax, int i) -> long {
    return std::min(2L * dims[ax], 2L * i * cell + cell) - std::max(0L, 2L * i * cell - cell);
  };
  std::vector<int32_t> cnt(n_gn + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    for (int e = 0; e < ne; ++e) {
      const int h = elem_geom(e, p, vert);
      int r[3][2];
      for (int ax = 0; ax < 3; ++ax) node_range(ax, p[ax], h, r[ax][0], r[ax][1]);
      for (int k = r[2][0]; k <= r[2][1]; ++k)
        for (int j = r[1][0]; j <= r[1][1]; ++j)
          for (int i = r[0][0]; i <= r[0][1]; ++i) {
            const long o = overlap2(0, i, p[0], h) * overlap2(1, j, p[1], h) * overlap2(2, k, p[2], h);
            if (o == 0) continue;
            const long g = ((long)k * NY + j) * NX + i;
            if (pass == 0) {
              ++cnt[g + 1];
            } else {
              celem[fill[g]] = e;
              cw[fill[g]++] = (double)o / ((double)box2(0, i) * box2(1, j) * box2(2, k));
            }
          }
    }
    if (pass == 0) {
      for (long g = 0; g < n_gn; ++g) cnt[g + 1] += cnt[g];
      celem.resize(cnt[n_gn]);
      cw.resize(cnt[n_gn]);
      fill.assign(cnt.begin(), cnt.end() - 1);
    }
  }
  // each grid node: the first element whose closed box holds it
  std::vector<int32_t> gnode(8 * n_gn, -1);
  std::vector<float> gw(8 * n_gn, 0.f);
  for (int e = 0; e < ne; ++e) {
    const int h = elem_geom(e, p, vert);
    const int gi0 = (p[0] + cell - 1) / cell, gi1 = (p[0] + h) / cell;
    const int gj0 = (p[1] + cell - 1) / cell, gj1 = (p[1] + h) / cell;
    const int gk0 = (p[2] + cell - 1) / cell, gk1 = (p[2] + h) / cell;
    for (int k = gk0; k <= gk1; ++k)
      for (int j = gj0; j <= gj1; ++j)
        for (int i = gi0; i <= gi1; ++i) {
          const long g = ((long)k * NY + j) * NX + i;
          if (gnode[8 * g] >= 0) continue;
          const double tx = (double)(i * cell - p[0]) / h, ty = (double)(j * cell - p[1]) / h,
                       tz = (double)(k * cell - p[2]) / h;
          for (int a = 0; a < 8; ++a) {
            gnode[8 * g + a] = vert[a];
            gw[8 * g + a] = (float)(((a & 1) ? tx : 1.0 - tx) * (((a >> 1) & 1) ? ty : 1.0 - ty) *
                                    ((a >> 2) ? tz : 1.0 - tz));
          }
        }
  }
  for (long g = 0; g < n_gn; ++g)
    if (gnode[8 * g] < 0) return ctx->fail(AMRTO_EINVAL, "grid: a grid node lies outside the mesh");
  auto up = [&](auto*& dst, const auto& v) -> hipError_t {
    if (dst) (void)hipFree(dst);
    dst = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(v[0]);
    hipError_t err = hipMalloc((void**)&dst, bytes);
    if (err == hipSuccess && !v.empty()) err = hipMemcpy(dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
    return err;
  };
  ctx->grid_cell = 0;
  AMRTO_HIP(up(ctx->d_cell_ptr, cnt));
  AMRTO_HIP(up(ctx->d_cell_elem, celem));
  AMRTO_HIP(up(ctx->d_cell_w, cw));
  AMRTO_HIP(up(ctx->d_gn_node, gnode));
  AMRTO_HIP(up(ctx->d_gn_w, gw));
  if (!ctx->uniform && !ctx->d_node_xyz) AMRTO_HIP(up(ctx->d_node_xyz, ctx->h_node_xyz));
  ctx->grid_cell = cell;
  return AMRTO_OK;
}

int amrto_grid_from_mesh(amrto_ctx* ctx, int32_t cell, const double* rho, const double* u, const double* u_ref,
                         double u_scale, float* rho_grid, float* u_grid) {
  if (!ctx) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_grid_from_mesh: no mesh");
  AMRTO_HIP(hipSetDevice(ctx->device));
  int rc = grid_maps(ctx, cell);
  if (rc) return rc;
  const long ngn = (long)(ctx->nx / cell + 1) * (ctx->ny / cell + 1) * (ctx->nz / cell + 1);
  if (rho && rho_grid)
    hipLaunchKernelGGL(k_grid_density, dim3((ngn + 255) / 256), dim3(256), 0, ctx->stream, rho, ctx->d_cell_ptr,
                       ctx->d_cell_elem, ctx->d_cell_w, (int)ngn, rho_grid);
  if (u && u_grid)
    hipLaunchKernelGGL(k_grid_sample, dim3((3 * ngn + 255) / 256), dim3(256), 0, ctx->stream, u, u_ref,
                       ctx->d_gn_node, ctx->d_gn_w, ngn, u_scale, u_grid);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

int amrto_grid_to_mesh(amrto_ctx* ctx, int32_t cell, const float* u_grid, double scale, double* u) {
  if (!ctx || !u_grid || !u) return AMRTO_EINVAL;
  if (!ctx->has_mesh) return ctx->fail(AMRTO_ESTATE, "amrto_grid_to_mesh: no mesh");
  AMRTO_HIP(hipSetDevice(ctx->device));
  int rc = grid_maps(ctx, cell);
  if (rc) return rc;
  hipLaunchKernelGGL(k_grid_interp, dim3((ctx->n_nodes + 255) / 256), dim3(256), 0, ctx->stream, u_grid,
                     ctx->uniform ? nullptr : ctx->d_node_xyz, ctx->n_nodes, cell, ctx->nx / cell, ctx->ny / cell,
                     ctx->nz / cell, scale, u, ctx->nx + 1, ctx->ny + 1);
  AMRTO_HIP(hipGetLastError());
  return AMRTO_OK;
}

}  // extern "C"
