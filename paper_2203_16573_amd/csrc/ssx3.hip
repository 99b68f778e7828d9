// Three-dimensional propagation F (source plane -> pressure traces on a
// receiver plane) and its exact transpose: the 3D form of the acoustic
// system of the Operators section with the source a density on the plane
// z = z_s (the closing remarks name 3D as the natural generalisation).
// Staggered grid: p on nodes, split p_x + p_y + p_z (kept on every cell), and
// v_x, v_y, v_z on the half nodes of their own axis; order 2 in time, 4 or
// 8 in space; the split-field absorbing layer of the 2D scheme applied per
// axis; planes sampled by linear interpolation in z, traces on grid nodes
// laterally (trace index iy * nx_traces + ix), injection its transpose.
// Constant density; FP64 or FP32 fields (the compute type is the storage
// type).
//
// Layout: each field is one [NZ][NY][NX] array, x fastest, no ghost cells
// (values outside the grid are read as zero).  The pressure is split into
// its three parts in the absorbing frame only: off the frame every layer
// factor is 1, the forward pressure is updated as one total, and the three
// parts' adjoints are equal and kept as one value.  One thread per ZW
// planes of a column (the z-stencil operands of those planes loaded once;
// one plane in k3_adj_v), 64 x 8 columns per workgroup; workgroups are
// dealt to the 8 XCDs round-robin, so the logical tile order gives each XCD
// a contiguous band of z planes, which it sweeps in order: the z-neighbour
// planes a stencil reads are then the ones its own L2 has just held.
//
// Forward step n: k3_vel (v^{n+1/2} from p^n), k3_pres (p^{n+1} from
// v^{n+1/2}, the source sample h[n] injected), then the receiver plane
// sampled (P[n] = R p^{n+1}).  Transposed step n (reverse order): the
// source-plane gather of the pressure adjoint (hbar[n]), k3_adj_v (the
// velocity adjoints: the previous step's layer scaling, then the transposed
// pressure updates), k3_adj_p (the pressure adjoints: layer scaling, the
// transposed velocity updates, and the recording of step n - 1 added).
#include "ssx3_internal.h"
#include "ssx_cell.h"

namespace ssx3 {
using ssx::acc;
using ssx::fmac;
using ssx::wst;

constexpr int BX = 64, BY = 8;
constexpr int ZW = 4;    // z planes per thread: k3_vel, k3_pres, k3_adj_p
constexpr int ZW_AV = 1;  // k3_adj_v (six stores per plane: one plane each)

// A thread's column and planes: logical tile of hardware block b (XCD bands
// of consecutive tiles, x tiles fastest, then y tiles, then chunks of Z z
// planes)
struct Cell {
  int x, y, z;
};
// the column (x, y) and the first of the thread's Z planes
template <int Z>
__device__ __forceinline__ Cell col_of(const Dims3& d) {
  const int n = (int)gridDim.x, b = (int)blockIdx.x;
  const int per = n >> 3, rem = n & 7, xcd = b & 7;
  const int t = xcd * per + (xcd < rem ? xcd : rem) + (b >> 3);
  const int tx = (d.NX + BX - 1) / BX, ty = (d.NY + BY - 1) / BY;
  const int zc = t / (tx * ty), r = t - zc * (tx * ty), yb = r / tx, xb = r - yb * tx;
  return {xb * BX + (int)threadIdx.x, yb * BY + (int)threadIdx.y, zc * Z};
}

template <typename T>
struct View {
  const T* a;
  int NZ, NY, NX;
  __device__ __forceinline__ T operator()(int z, int y, int x) const {
    return (z < 0 || z >= NZ || y < 0 || y >= NY || x < 0 || x >= NX)
               ? T(0)
               : a[((long long)z * NY + y) * NX + x];
  }
};

// layer factors: per axis (z, y, x) four arrays a_node, b_node, a_half,
// b_half of the axis length, one after another
template <typename T>
struct Fac {
  const T* f;
  int NZ, NY, NX;
  __device__ __forceinline__ const T* ax(int axis) const {
    return axis == 0 ? f : (axis == 1 ? f + 4 * NZ : f + 4 * NZ + 4 * NY);
  }
  __device__ __forceinline__ T an(int axis, int i) const { return ax(axis)[i]; }
  __device__ __forceinline__ T bn(int axis, int i) const {
    return ax(axis)[(axis == 0 ? NZ : axis == 1 ? NY : NX) + i];
  }
  __device__ __forceinline__ T ah(int axis, int i) const {
    return ax(axis)[2 * (axis == 0 ? NZ : axis == 1 ? NY : NX) + i];
  }
  __device__ __forceinline__ T bh(int axis, int i) const {
    return ax(axis)[3 * (axis == 0 ? NZ : axis == 1 ? NY : NX) + i];
  }
};

// off the absorbing frame, where every layer factor is 1 and the pressure
// is not split
__device__ __forceinline__ bool inner(const Dims3& d, int z, int y, int x) {
  return z >= d.L && z < d.NZ - d.L && y >= d.L && y < d.NY - d.L && x >= d.L && x < d.NX - d.L;
}

// the interpolation weight with which cell (z, y, x) enters plane pl (zero
// off the plane), and the trace index there
__device__ __forceinline__ double plane_w(const Plane3& pl, int z, int y, int x, int& tr) {
  if (y < pl.y0 || y >= pl.y0 + pl.ny || x < pl.x0 || x >= pl.x0 + pl.nx) return 0.0;
  tr = (y - pl.y0) * pl.nx + (x - pl.x0);
  double w = 0.0;
  if (z == pl.r0) w += pl.w0;
  if (pl.r1 >= 0 && z == pl.r1) w += pl.w1;
  return w;
}

// Each thread takes Z consecutive planes of its column; the 2K + Z - 1
// values the z-stencils of those planes read are loaded once, in w.
template <int K, typename T, int Z>
__global__ __launch_bounds__(BX* BY) void k3_vel(Fields3<T> f, Dims3 d, const T* fac, T cb,
                                                 Plane3 fpl, const T* ftr) {
  const Cell cc = col_of<Z>(d);
  const int x = cc.x, y = cc.y, z0 = cc.z;
  if (x >= d.NX || y >= d.NY) return;
  const View<T> p{f.p, d.NZ, d.NY, d.NX};
  const Fac<T> F{fac, d.NZ, d.NY, d.NX};
  T w[2 * K + Z - 1];  // p at planes z0 + 1 - K ..
#pragma unroll
  for (int j = 0; j < 2 * K + Z - 1; ++j) w[j] = p(z0 + 1 - K + j, y, x);
#pragma unroll
  for (int j = 0; j < Z; ++j) {
    const int z = z0 + j;
    if (z >= d.NZ) break;
    const long long o = ((long long)z * d.NY + y) * d.NX + x;
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
      const T c = wst<K, T>(m - 1);
      gx = acc(gx, c, p(z, y, x + m), p(z, y, x + 1 - m));
      gy = acc(gy, c, p(z, y + m, x), p(z, y + 1 - m, x));
      gz = acc(gz, c, w[j + K - 1 + m], w[j + K - m]);
    }
    if (ftr) {  // a normal load on plane fpl (v_z nodes): D_z^+ p - E_f f
      int tr = 0;
      const double wt = plane_w(fpl, z, y, x, tr);
      if (wt != 0.0) gz = gz - T(wt) * ftr[tr];
    }
    f.vx[o] = fmac(F.ah(2, x), f.vx[o], -(F.bh(2, x) * cb) * gx);
    f.vy[o] = fmac(F.ah(1, y), f.vy[o], -(F.bh(1, y) * cb) * gy);
    f.vz[o] = fmac(F.ah(0, z), f.vz[o], -(F.bh(0, z) * cb) * gz);
  }
}

template <int K, typename T, int Z>
__global__ __launch_bounds__(BX* BY) void k3_pres(Fields3<T> f, Dims3 d, const T* fac,
                                                  const T* ck, Plane3 src, const T* htr) {
  const Cell cc = col_of<Z>(d);
  const int x = cc.x, y = cc.y, z0 = cc.z;
  if (x >= d.NX || y >= d.NY) return;
  const View<T> vx{f.vx, d.NZ, d.NY, d.NX}, vy{f.vy, d.NZ, d.NY, d.NX},
      vz{f.vz, d.NZ, d.NY, d.NX};
  const Fac<T> F{fac, d.NZ, d.NY, d.NX};
  T w[2 * K + Z - 1];  // v_z at planes z0 - K ..
#pragma unroll
  for (int j = 0; j < 2 * K + Z - 1; ++j) w[j] = vz(z0 - K + j, y, x);
#pragma unroll
  for (int j = 0; j < Z; ++j) {
    const int z = z0 + j;
    if (z >= d.NZ) break;
    const long long o = ((long long)z * d.NY + y) * d.NX + x;
    T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
      const T c = wst<K, T>(m - 1);
      dx = acc(dx, c, vx(z, y, x + m - 1), vx(z, y, x - m));
      dy = acc(dy, c, vy(z, y + m - 1, x), vy(z, y - m, x));
      dz = acc(dz, c, w[j + K + m - 1], w[j + K - m]);
    }
    if (htr) {
      int tr = 0;
      const double wt = plane_w(src, z, y, x, tr);
      if (wt != 0.0) dz = dz - T(wt) * htr[tr];
    }
    const T k = ck[o];
    if (inner(d, z, y, x)) {
      f.p[o] = fmac(-k, (dx + dy) + dz, f.p[o]);
      continue;
    }
    const T px = fmac(F.an(2, x), f.px[o], -(F.bn(2, x) * k) * dx);
    const T py = fmac(F.an(1, y), f.py[o], -(F.bn(1, y) * k) * dy);
    const T pz = fmac(F.an(0, z), f.pz[o], -(F.bn(0, z) * k) * dz);
    f.px[o] = px;
    f.py[o] = py;
    f.pz[o] = pz;
    f.p[o] = (px + py) + pz;
  }
}

// Transposed pressure updates: the velocity adjoints take the layer scaling
// pending from the previous transposed step (a_half v~) and the v_z
// recording of this step (u_a stored with each updated v~_a), then
//   v~_a += sum_m c_m (q_a[i+m] - q_a[i+1-m]),  q_a = b_node,a Ck p~_a,
// the transpose of p_a -= b_node,a Ck D_a^- v_a (D^- = -(D^+)^T).
template <int K, typename T, int Z>
__global__ __launch_bounds__(BX* BY) void k3_adj_v(Fields3<T> f, Dims3 d, const T* fac, T cb,
                                                   Plane3 vpl, const T* vtr) {
  const Cell cc = col_of<Z>(d);
  const int x = cc.x, y = cc.y, z0 = cc.z;
  if (x >= d.NX || y >= d.NY) return;
  const Fac<T> F{fac, d.NZ, d.NY, d.NX};
  // q_a = b_node,a Ck p~_a at the neighbouring nodes, as the kernel that
  // last updated p~_a stored it (zero outside the grid)
  const View<T> qx{f.qx, d.NZ, d.NY, d.NX}, qy{f.qy, d.NZ, d.NY, d.NX},
      qz{f.qz, d.NZ, d.NY, d.NX};
  T w[2 * K + Z - 1];  // q_z at planes z0 + 1 - K ..
#pragma unroll
  for (int j = 0; j < 2 * K + Z - 1; ++j) w[j] = qz(z0 + 1 - K + j, y, x);
#pragma unroll
  for (int j = 0; j < Z; ++j) {
    const int z = z0 + j;
    if (z >= d.NZ) break;
    const long long o = ((long long)z * d.NY + y) * d.NX + x;
    T sx = T(0), sy_ = T(0), sz_ = T(0);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
      const T c = wst<K, T>(m - 1);
      sx = acc(sx, c, qx(z, y, x + m), qx(z, y, x + 1 - m));
      sy_ = acc(sy_, c, qy(z, y + m, x), qy(z, y + 1 - m, x));
      sz_ = acc(sz_, c, w[j + K - 1 + m], w[j + K - m]);
    }
    // the v_z recording of this step (V = R v_z) enters after the scaling
    T rv = T(0);
    if (vtr) {
      int tr = 0;
      const double wt = plane_w(vpl, z, y, x, tr);
      if (wt != 0.0) rv = T(wt) * vtr[tr];
    }
    const T vbx = F.ah(2, x) * f.vx[o] + sx;
    const T vby = F.ah(1, y) * f.vy[o] + sy_;
    const T vbz = (F.ah(0, z) * f.vz[o] + rv) + sz_;
    f.vx[o] = vbx;
    f.vy[o] = vby;
    f.vz[o] = vbz;
    f.ux[o] = (F.bh(2, x) * cb) * vbx;
    f.uy[o] = (F.bh(1, y) * cb) * vby;
    f.uz[o] = (F.bh(0, z) * cb) * vbz;
  }
}

// Transposed velocity updates (q_a stored with each updated p~_a):
// p~_a <- a_node,a p~_a + t, with
//   t = sum_a sum_m c_m (u_a[i+m-1] - u_a[i-m]),  u_a = b_half,a Cb v~_a
// (the transpose of v_a -= b_half,a Cb D_a^+ p, p = p_x + p_y + p_z, taken
// by all three parts), then the recording of step n - 1 (P = R p) added to
// each part.
template <int K, typename T, int Z>
__global__ __launch_bounds__(BX* BY) void k3_adj_p(Fields3<T> f, Dims3 d, const T* fac,
                                                   const T* ck, T cb, Plane3 rec, const T* rtr) {
  const Cell cc = col_of<Z>(d);
  const int x = cc.x, y = cc.y, z0 = cc.z;
  if (x >= d.NX || y >= d.NY) return;
  (void)cb;  // the b_half Cb factors are in u, as k3_adj_v stored it
  const Fac<T> F{fac, d.NZ, d.NY, d.NX};
  // u_a = b_half,a Cb v~_a at the neighbouring half nodes, as k3_adj_v
  // stored it (zero outside the grid)
  const View<T> ux{f.ux, d.NZ, d.NY, d.NX}, uy{f.uy, d.NZ, d.NY, d.NX},
      uz{f.uz, d.NZ, d.NY, d.NX};
  T w[2 * K + Z - 1];  // u_z at planes z0 - K ..
#pragma unroll
  for (int j = 0; j < 2 * K + Z - 1; ++j) w[j] = uz(z0 - K + j, y, x);
#pragma unroll
  for (int j = 0; j < Z; ++j) {
    const int z = z0 + j;
    if (z >= d.NZ) break;
    const long long o = ((long long)z * d.NY + y) * d.NX + x;
    T tx = T(0), ty = T(0), tz = T(0);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
      const T c = wst<K, T>(m - 1);
      tx = acc(tx, c, ux(z, y, x + m - 1), ux(z, y, x - m));
      ty = acc(ty, c, uy(z, y + m - 1, x), uy(z, y - m, x));
      tz = acc(tz, c, w[j + K + m - 1], w[j + K - m]);
    }
    const T t = (tx + ty) + tz;
    T r = T(0);
    if (rtr) {
      int tr = 0;
      const double wt = plane_w(rec, z, y, x, tr);
      if (wt != 0.0) r = T(wt) * rtr[tr];
    }
    const T k = ck[o];
    if (inner(d, z, y, x)) {
      const T pb = (f.p[o] + t) + r;
      f.p[o] = pb;
      f.qx[o] = (F.bn(2, x) * k) * pb;
      f.qy[o] = (F.bn(1, y) * k) * pb;
      f.qz[o] = (F.bn(0, z) * k) * pb;
      continue;
    }
    const T pbx = fmac(F.an(2, x), f.px[o], t) + r;
    const T pby = fmac(F.an(1, y), f.py[o], t) + r;
    const T pbz = fmac(F.an(0, z), f.pz[o], t) + r;
    f.px[o] = pbx;
    f.py[o] = pby;
    f.pz[o] = pbz;
    f.qx[o] = (F.bn(2, x) * k) * pbx;
    f.qy[o] = (F.bn(1, y) * k) * pby;
    f.qz[o] = (F.bn(0, z) * k) * pbz;
  }
}

// the recording's transpose alone (the first transposed step): each part
// of the pressure adjoint += R^T r
template <typename T>
__global__ void k3_spread(Fields3<T> f, Dims3 d, Plane3 pl, const T* fac, const T* ck,
                          const T* tr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * pl.ny * pl.nx) return;
  const int row = i / (pl.ny * pl.nx), t = i - row * (pl.ny * pl.nx);
  if (row == 1 && pl.r1 < 0) return;
  const int z = row ? pl.r1 : pl.r0, y = pl.y0 + t / pl.nx, x = pl.x0 + t % pl.nx;
  const T w = T(row ? pl.w1 : pl.w0);
  const long long o = ((long long)z * d.NY + y) * d.NX + x;
  const T v = w * tr[t];
  const Fac<T> F{fac, d.NZ, d.NY, d.NX};
  const T k = ck[o];
  if (inner(d, z, y, x)) {
    const T pb = f.p[o] + v;
    f.p[o] = pb;
    f.qx[o] = (F.bn(2, x) * k) * pb;
    f.qy[o] = (F.bn(1, y) * k) * pb;
    f.qz[o] = (F.bn(0, z) * k) * pb;
    return;
  }
  f.px[o] += v;
  f.py[o] += v;
  f.pz[o] += v;
  f.qx[o] = (F.bn(2, x) * k) * f.px[o];
  f.qy[o] = (F.bn(1, y) * k) * f.py[o];
  f.qz[o] = (F.bn(0, z) * k) * f.pz[o];
}

// plane gather: out[t] = sum_rows w s v, with (MODE 0) v = p, s = 1; (1)
// the pressure-source slot of the transpose, v = the z part's adjoint, s =
// b_node,z Ck; (2) v = v_z, s = 1; (3) the normal-load slot of the
// transpose, v = v_z's adjoint, s = b_half,z Cb
template <typename T, int MODE>
__global__ void k3_gather(Fields3<T> f, Dims3 d, Plane3 pl, const T* fac, const T* ck, T cb,
                          T* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pl.ny * pl.nx) return;
  const int y = pl.y0 + t / pl.nx, x = pl.x0 + t % pl.nx;
  (void)fac;  // the scaled values (modes 1, 3) are read as the step kernels
  (void)ck;   // stored them
  (void)cb;
  auto val = [&](int z) {
    const long long o = ((long long)z * d.NY + y) * d.NX + x;
    if (MODE == 0) return f.p[o];
    if (MODE == 2) return f.vz[o];
    if (MODE == 3) return f.uz[o];  // b_half,z Cb v~_z, as stored
    return f.qz[o];  // (MODE 1) b_node,z Ck p~_z, as stored
  };
  T s = T(pl.w0) * val(pl.r0);
  if (pl.r1 >= 0) s = s + T(pl.w1) * val(pl.r1);
  out[t] = s;
}

// ---------------------------------------------------------------------------

static dim3 columns(const Dims3& d, int z) {
  return dim3((unsigned)(((d.NX + BX - 1) / BX) * ((d.NY + BY - 1) / BY) *
                         ((d.NZ + z - 1) / z)));
}

template <typename T>
static hipError_t step_t(int order, bool adj, const Fields3<T>& f, const Dims3& d, const T* fac,
                         const T* ck, T cb, const Plane3& pl, const T* tr, const Plane3& pl2,
                         const T* tr2, hipStream_t s) {
  const dim3 gc = columns(d, ZW), gv = columns(d, ZW_AV), b(BX, BY);
  if (d.NZ < 1 || d.NZ > 65535) return hipErrorInvalidValue;
  if (order == 4) {
    if (!adj) {
      hipLaunchKernelGGL((k3_vel<2, T, ZW>), gc, b, 0, s, f, d, fac, cb, pl2, tr2);
      hipLaunchKernelGGL((k3_pres<2, T, ZW>), gc, b, 0, s, f, d, fac, ck, pl, tr);
    } else {
      hipLaunchKernelGGL((k3_adj_v<2, T, ZW_AV>), gv, b, 0, s, f, d, fac, cb, pl2, tr2);
      hipLaunchKernelGGL((k3_adj_p<2, T, ZW>), gc, b, 0, s, f, d, fac, ck, cb, pl, tr);
    }
  } else if (order == 8) {
    if (!adj) {
      hipLaunchKernelGGL((k3_vel<4, T, ZW>), gc, b, 0, s, f, d, fac, cb, pl2, tr2);
      hipLaunchKernelGGL((k3_pres<4, T, ZW>), gc, b, 0, s, f, d, fac, ck, pl, tr);
    } else {
      hipLaunchKernelGGL((k3_adj_v<4, T, ZW_AV>), gv, b, 0, s, f, d, fac, cb, pl2, tr2);
      hipLaunchKernelGGL((k3_adj_p<4, T, ZW>), gc, b, 0, s, f, d, fac, ck, cb, pl, tr);
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch3_step(bool f64, int order, bool adj, const void* fields, const Dims3& d,
                        const void* fac, const void* ck, double cb, const Plane3& pl,
                        const void* tr, const Plane3& pl2, const void* tr2, hipStream_t s) {
  if (f64)
    return step_t<double>(order, adj, fields3<double>(fields, d), d, (const double*)fac,
                          (const double*)ck, cb, pl, (const double*)tr, pl2,
                          (const double*)tr2, s);
  return step_t<float>(order, adj, fields3<float>(fields, d), d, (const float*)fac,
                       (const float*)ck, (float)cb, pl, (const float*)tr, pl2,
                       (const float*)tr2, s);
}

hipError_t launch3_spread(bool f64, const void* fields, const Dims3& d, const Plane3& pl,
                          const void* fac, const void* ck, const void* tr, hipStream_t s) {
  const int n = 2 * pl.ny * pl.nx;
  const dim3 g((n + 255) / 256), b(256);
  if (f64)
    hipLaunchKernelGGL((k3_spread<double>), g, b, 0, s, fields3<double>(fields, d), d, pl,
                       (const double*)fac, (const double*)ck, (const double*)tr);
  else
    hipLaunchKernelGGL((k3_spread<float>), g, b, 0, s, fields3<float>(fields, d), d, pl,
                       (const float*)fac, (const float*)ck, (const float*)tr);
  return hipGetLastError();
}

template <typename T>
static void gather_t(int mode, const Fields3<T>& f, const Dims3& d, const Plane3& pl,
                     const T* fac, const T* ck, T cb, T* out, hipStream_t s) {
  const int n = pl.ny * pl.nx;
  const dim3 g((n + 255) / 256), b(256);
  switch (mode) {
    case 0: hipLaunchKernelGGL((k3_gather<T, 0>), g, b, 0, s, f, d, pl, fac, ck, cb, out); break;
    case 1: hipLaunchKernelGGL((k3_gather<T, 1>), g, b, 0, s, f, d, pl, fac, ck, cb, out); break;
    case 2: hipLaunchKernelGGL((k3_gather<T, 2>), g, b, 0, s, f, d, pl, fac, ck, cb, out); break;
    default: hipLaunchKernelGGL((k3_gather<T, 3>), g, b, 0, s, f, d, pl, fac, ck, cb, out);
  }
}

hipError_t launch3_gather(bool f64, int mode, const void* fields, const Dims3& d,
                          const Plane3& pl, const void* fac, const void* ck, double cb,
                          void* out, hipStream_t s) {
  if (mode < 0 || mode > 3) return hipErrorInvalidValue;
  if (f64)
    gather_t<double>(mode, fields3<double>(fields, d), d, pl, (const double*)fac,
                     (const double*)ck, cb, (double*)out, s);
  else
    gather_t<float>(mode, fields3<float>(fields, d), d, pl, (const float*)fac,
                    (const float*)ck, (float)cb, (float*)out, s);
  return hipGetLastError();
}

// y[n][t] = sc s_t x[n][t] over nt steps of nt_tr traces: s_t = dist_t (op
// 0, A), dist_t^2 (1, A^T A) or (1 + a^2 dist_t^2)^(-1/2) (2, D); dist: the
// lateral distance of each trace from the physical point (FP64)
template <typename T>
__global__ void k3_diag(int op, double a, double sc, const double* dist, const T* x, T* y,
                        long long n, int ntr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dd = dist[i % ntr];
  const double f = op == 0 ? dd : (op == 1 ? dd * dd : 1.0 / sqrt(1.0 + (a * dd) * (a * dd)));
  y[i] = T(sc * f * (double)x[i]);
}

// y = x + a z (FP64 a)
template <typename T>
__global__ void k3_axpy(T* y, const T* x, double a, const T* z, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = T((double)x[i] + a * (double)z[i]);
}

hipError_t launch3_diag(bool f64, int op, double a, double sc, const double* dist, const void* x,
                        void* y, long long n, int ntr, hipStream_t s) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (f64)
    hipLaunchKernelGGL((k3_diag<double>), g, b, 0, s, op, a, sc, dist, (const double*)x,
                       (double*)y, n, ntr);
  else
    hipLaunchKernelGGL((k3_diag<float>), g, b, 0, s, op, a, sc, dist, (const float*)x,
                       (float*)y, n, ntr);
  return hipGetLastError();
}

hipError_t launch3_axpy(bool f64, void* y, const void* x, double a, const void* z, long long n,
                        hipStream_t s) {
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (f64)
    hipLaunchKernelGGL((k3_axpy<double>), g, b, 0, s, (double*)y, (const double*)x, a,
                       (const double*)z, n);
  else
    hipLaunchKernelGGL((k3_axpy<float>), g, b, 0, s, (float*)y, (const float*)x, a,
                       (const float*)z, n);
  return hipGetLastError();
}

// <x, y> in FP64: 256 workgroups of 256 threads each sum a fixed strided
// share and fold it in LDS in a fixed order, then one workgroup folds the
// 256 partial sums the same way (bitwise deterministic)
constexpr int DOT_BLOCKS = 256;

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

template <typename T>
__global__ __launch_bounds__(256) void k3_dot_partial(const T* x, const T* y, long long n,
                                                      double* partial) {
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += 256LL * DOT_BLOCKS)
    acc += (double)x[i] * (double)y[i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k3_dot_final(const double* partial, double* out) {
  const double s = block_sum(partial[threadIdx.x]);
  if (threadIdx.x == 0) out[0] = s;
}

hipError_t launch3_dot(bool f64, const void* x, const void* y, long long n, double* partial,
                       double* out, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL((k3_dot_partial<double>), dim3(DOT_BLOCKS), dim3(256), 0, s,
                       (const double*)x, (const double*)y, n, partial);
  else
    hipLaunchKernelGGL((k3_dot_partial<float>), dim3(DOT_BLOCKS), dim3(256), 0, s,
                       (const float*)x, (const float*)y, n, partial);
  hipLaunchKernelGGL(k3_dot_final, dim3(1), dim3(256), 0, s, partial, out);
  return hipGetLastError();
}

}  // namespace ssx3
