// C ABI of libcprrtc.so: argument checking, handle lifecycle (robot and
// scene copies in HBM), error mapping and kernel dispatch.  Every exported
// function catches everything and returns a status code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cprrtc.h"
#include "device.h"
#include "handles.h"
#include "kernels.h"

using namespace cprrtc;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(CP_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Rotation entries within 1e-6 of 0 or +-1 are stored as those values (cos
// and sin of multiples of pi/2 land a few 1e-8 off in float), so that a
// kernel compiled with the robot's constants can drop the terms they zero.
float snap_unit(float v) {
  if (std::fabs(v) < 1e-6f) return 0.0f;
  if (std::fabs(v - 1.0f) < 1e-6f) return 1.0f;
  if (std::fabs(v + 1.0f) < 1e-6f) return -1.0f;
  return v;
}

void copy34(float* dst, const double* m16) {
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 4; ++c) dst[4 * i + c] = (float)m16[4 * i + c];
}

int make_constraint(const cp_constraint* c, const cp_robot* robot, ConDev* out) {
  std::memset(out, 0, sizeof *out);
  if (!c) {
    out->kind = KIND_NONE;
    return CP_OK;
  }
  if (c->kind < CP_CON_NONE || c->kind > CP_CON_REL_POSE)
    return fail(CP_E_ARG, "constraint kind %d unknown", c->kind);
  out->kind = c->kind;
  for (int i = 0; i < 6; ++i) out->mask[i] = c->mask[i] ? 1.0f : 0.0f;
  if (c->kind == CP_CON_POSE) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) out->Rt[3 * i + k] = (float)c->frame[4 * k + i];
    for (int i = 0; i < 3; ++i) out->pc[i] = (float)c->frame[4 * i + 3];
    for (int i = 0; i < 6; ++i) out->target[i] = (float)c->target[i];
  } else if (c->kind == CP_CON_REL_POSE) {
    if (robot->host.n_chains != 2)
      return fail(CP_E_ARG, "relative-pose constraint needs a two-chain robot");
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) out->Rt[3 * i + k] = (float)c->rel_target[4 * k + i];
    for (int i = 0; i < 3; ++i) out->target[i] = (float)c->rel_target[4 * i + 3];
  }
  return CP_OK;
}

}  // namespace

namespace cprrtc {
int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}
int api_hip_fail(hipError_t e, const char* what) { return hip_fail(e, what); }
int api_constraint(const cp_constraint* c, const cp_robot* robot, ConDev* out) {
  return make_constraint(c, robot, out);
}
}  // namespace cprrtc

extern "C" {

const char* cp_last_error(void) { return g_error.c_str(); }

void cp_proj_params_default(cp_proj_params* p) {
  if (!p) return;
  p->W = 64;
  p->max_iters = 32;
  p->tau = 0.05;
  p->tau_sm = 0.025;
  p->tau_task = 1e-3;
  p->alpha = 1.0;
  p->lambda = 1e-2;
  p->sphere_batch = 8;
  p->variant = CP_PROJECT_PARALLEL;
}

namespace {

// Sphere centres (double, world) of a robot description at the home
// configuration (every joint at 0 clamped into its limits), by the modified
// DH convention: per joint, rotate about x by alpha, move a along x, rotate
// about z by theta, move d along z.
std::vector<double> home_centres(const cp_robot_desc* d) {
  std::vector<double> frames((size_t)d->dof * 16);
  for (int c = 0; c < d->n_chains; ++c) {
    double T[16];
    std::memcpy(T, d->base + 16 * c, sizeof T);
    for (int j = 0; j < d->dof; ++j) {
      if (d->joint_chain[j] != c) continue;
      const double q = std::min(std::max(0.0, d->q_lo[j]), d->q_hi[j]);
      const bool pri = d->joint_type[j] == CP_PRISMATIC;
      const double th = d->theta[j] + (pri ? 0.0 : q), dd = d->d[j] + (pri ? q : 0.0);
      const double ca = std::cos(d->alpha[j]), sa = std::sin(d->alpha[j]);
      const double ct = std::cos(th), st = std::sin(th);
      // the joint's local transform (rows of the 3x4 part)
      const double L[12] = {ct, -st, 0.0, d->a[j],
                            ca * st, ca * ct, -sa, -sa * dd,
                            sa * st, sa * ct, ca, ca * dd};
      double N[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1};
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 4; ++k) {
          double v = k == 3 ? T[4 * r + 3] : 0.0;
          for (int m = 0; m < 3; ++m) v += T[4 * r + m] * L[4 * m + k];
          N[4 * r + k] = v;
        }
      std::memcpy(T, N, sizeof T);
      std::memcpy(&frames[(size_t)j * 16], T, sizeof T);
    }
  }
  std::vector<double> xyz((size_t)d->n_spheres * 3);
  for (int s = 0; s < d->n_spheres; ++s) {
    const double* T = &frames[(size_t)d->sphere_link[s] * 16];
    const double* l = d->sphere + 4 * s;
    for (int r = 0; r < 3; ++r)
      xyz[3 * s + r] = T[4 * r] * l[0] + T[4 * r + 1] * l[1] + T[4 * r + 2] * l[2] + T[4 * r + 3];
  }
  return xyz;
}

// Self-collision pairs (description order, s < t, lexicographic): spheres on
// links of different chains, or of one chain at least two joints apart, that
// are clear by more than kSelfHomeClearance at the home configuration
// (pairs that overlap there touch across a joint by construction).
constexpr double kSelfHomeClearance = 1e-3;
std::vector<int32_t> self_pairs(const cp_robot_desc* d) {
  const std::vector<double> c = home_centres(d);
  std::vector<int32_t> out;
  for (int s = 0; s < d->n_spheres; ++s)
    for (int t = s + 1; t < d->n_spheres; ++t) {
      const int ls = d->sphere_link[s], lt = d->sphere_link[t];
      const bool rule = d->joint_chain[ls] != d->joint_chain[lt] || std::abs(ls - lt) >= 2;
      if (!rule) continue;
      const double dx = c[3 * s] - c[3 * t], dy = c[3 * s + 1] - c[3 * t + 1],
                   dz = c[3 * s + 2] - c[3 * t + 2];
      const double sd = std::sqrt(dx * dx + dy * dy + dz * dz) - d->sphere[4 * s + 3] -
                        d->sphere[4 * t + 3];
      if (sd > kSelfHomeClearance) {
        out.push_back(s);
        out.push_back(t);
      }
    }
  return out;
}

}  // namespace

int cp_robot_create(const cp_robot_desc* d, cp_robot** out) {
  try {
    if (!d || !out) return fail(CP_E_ARG, "cp_robot_create: NULL argument");
    *out = nullptr;
    if (d->dof < 1 || d->dof > kMaxDof) return fail(CP_E_UNSUPPORTED, "dof %d not in 1..%d", d->dof, kMaxDof);
    if (d->n_chains < 1 || d->n_chains > kMaxChains)
      return fail(CP_E_UNSUPPORTED, "n_chains %d not in 1..%d", d->n_chains, kMaxChains);
    if (!d->joint_type || !d->joint_chain || !d->alpha || !d->a || !d->d || !d->theta || !d->q_lo ||
        !d->q_hi || !d->base || !d->tool || !d->sphere_link || !d->sphere)
      return fail(CP_E_ARG, "cp_robot_create: NULL array");
    if (d->n_spheres < 1 || d->n_spheres > kMaxSpheres)
      return fail(CP_E_UNSUPPORTED, "n_spheres %d not in 1..%d", d->n_spheres, kMaxSpheres);
    RobotDev h;
    std::memset(&h, 0, sizeof h);
    h.dof = d->dof;
    h.n_chains = d->n_chains;
    int prev = 0;
    std::vector<int> count(d->n_chains, 0);
    for (int j = 0; j < d->dof; ++j) {
      const int c = d->joint_chain[j];
      if (c < 0 || c >= d->n_chains || c < prev)
        return fail(CP_E_ARG, "joint_chain must be non-decreasing in [0, n_chains)");
      prev = c;
      count[c]++;
      if (d->joint_type[j] != CP_REVOLUTE && d->joint_type[j] != CP_PRISMATIC)
        return fail(CP_E_ARG, "joint %d: unknown type %d", j, d->joint_type[j]);
      if (!(d->q_lo[j] <= d->q_hi[j])) return fail(CP_E_ARG, "joint %d: q_lo > q_hi", j);
      h.ca[j] = snap_unit((float)std::cos(d->alpha[j]));
      h.sa[j] = snap_unit((float)std::sin(d->alpha[j]));
      h.a[j] = (float)d->a[j];
      h.d0[j] = (float)d->d[j];
      h.th0[j] = (float)d->theta[j];
      h.lo[j] = (float)d->q_lo[j];
      h.hi[j] = (float)d->q_hi[j];
      h.prismatic[j] = d->joint_type[j] == CP_PRISMATIC;
      h.short_angle[j] = !h.prismatic[j] && std::fabs(h.lo[j] + h.th0[j]) <= 3.2f &&
                         std::fabs(h.hi[j] + h.th0[j]) <= 3.2f;
    }
    h.chain_begin[0] = 0;
    for (int c = 0; c < d->n_chains; ++c) {
      if (count[c] == 0) return fail(CP_E_ARG, "chain %d has no joints", c);
      h.chain_begin[c + 1] = h.chain_begin[c] + count[c];
    }
    for (int c = d->n_chains + 1; c <= kMaxChains; ++c) h.chain_begin[c] = d->dof;
    for (int c = 0; c < d->n_chains; ++c) {
      copy34(h.base[c], d->base + 16 * c);
      copy34(h.tool[c], d->tool + 16 * c);
      for (int i = 0; i < 12; ++i)
        if (i % 4 != 3) {
          h.base[c][i] = snap_unit(h.base[c][i]);
          h.tool[c][i] = snap_unit(h.tool[c][i]);
        }
    }
    // spheres grouped by the joint frame that carries them
    std::vector<int> order(d->n_spheres);
    for (int s = 0; s < d->n_spheres; ++s) {
      const int l = d->sphere_link[s];
      if (l < 0 || l >= d->dof) return fail(CP_E_ARG, "sphere %d: link %d out of range", s, l);
      if (!(d->sphere[4 * s + 3] > 0.0)) return fail(CP_E_ARG, "sphere %d: radius must be > 0", s);
      order[s] = s;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return d->sphere_link[x] < d->sphere_link[y]; });
    std::vector<float4> sph(d->n_spheres);
    for (int s = 0; s < d->n_spheres; ++s) {
      const double* src = d->sphere + 4 * order[s];
      sph[s] = make_float4((float)src[0], (float)src[1], (float)src[2], (float)src[3]);
    }
    for (int j = 0; j <= d->dof; ++j) h.sph_begin[j] = 0;
    for (int s = 0; s < d->n_spheres; ++s) h.sph_begin[d->sphere_link[s] + 1]++;
    for (int j = 0; j < d->dof; ++j) h.sph_begin[j + 1] += h.sph_begin[j];
    for (int j = d->dof + 1; j <= kMaxDof; ++j) h.sph_begin[j] = h.sph_begin[d->dof];
    h.n_spheres = d->n_spheres;

    cp_robot* r = new (std::nothrow) cp_robot;
    if (!r) return fail(CP_E_ARG, "out of host memory");
    r->host = h;
    // self-collision pairs, kept in description order for cp_robot_self_pairs
    // and as positions in the link-grouped sphere array for the kernels
    r->self_pairs = self_pairs(d);
    std::vector<int> rank(d->n_spheres);
    for (int s = 0; s < d->n_spheres; ++s) rank[order[s]] = s;
    const int n_pairs = (int)r->self_pairs.size() / 2;
    // The kernel's list: each checked pair filed under its first sphere s,
    // a sphere's pairs in groups of kGroup records (the last group filled up
    // with never-hitting records of the same s), group g at entries
    // (g / 16) kSelfPad + g % 16 + 16 u, so the 16 lanes of a row take 16
    // groups per loop trip and each reads its c_s once per group; then
    // never-hitting records up to a multiple of kSelfPad, and kSelfPad more
    // that the kernel reads ahead.
    constexpr int kGroup = kSelfPad / 16;
    const float never = -1.0f;   // d^2 <= -1 never holds
    int never_bits;
    std::memcpy(&never_bits, &never, sizeof never_bits);
    std::vector<int2> dev_pairs(n_pairs);
    std::vector<std::vector<int2>> by_s(d->n_spheres);
    for (int i = 0; i < n_pairs; ++i) {
      const int s0 = rank[r->self_pairs[2 * i]], t0 = rank[r->self_pairs[2 * i + 1]];
      dev_pairs[i] = make_int2(s0, t0);
      const double reach = (double)sph[s0].w + (double)sph[t0].w;
      const float reach2 = (float)(reach * reach);
      int bits;
      std::memcpy(&bits, &reach2, sizeof bits);
      by_s[s0].push_back(make_int2(s0 | (t0 << 16), bits));   // positions < kMaxSpheres <= 2^16
    }
    std::vector<int2> groups;   // kGroup records per group
    for (int s = 0; s < d->n_spheres; ++s) {
      const std::vector<int2>& v = by_s[s];
      for (size_t k = 0; k < v.size(); k += kGroup)
        for (int u = 0; u < kGroup; ++u)
          groups.push_back(k + u < v.size() ? v[k + u] : make_int2(s | (s << 16), never_bits));
    }
    const int n_groups = (int)groups.size() / kGroup;
    const int n_cc = (n_groups + 15) / 16 * kSelfPad;
    const int n_padded = n_cc + kSelfPad;
    std::vector<int2> cc_pairs(n_padded, make_int2(0, never_bits));
    for (int g = 0; g < n_groups; ++g)
      for (int u = 0; u < kGroup; ++u)
        cc_pairs[(g / 16) * kSelfPad + g % 16 + 16 * u] = groups[(size_t)g * kGroup + u];
    r->n_cc = n_cc;
    std::vector<int2> sph_map(d->n_spheres);
    for (int s = 0; s < d->n_spheres; ++s) sph_map[s] = make_int2(rank[s], d->sphere_link[s]);
    hipError_t e = hipMalloc((void**)&r->dev, sizeof(RobotDev));
    if (e == hipSuccess) e = hipMalloc((void**)&r->spheres, sizeof(float4) * sph.size());
    if (e == hipSuccess) e = hipMalloc((void**)&r->sph_map, sizeof(int2) * sph_map.size());
    if (e == hipSuccess)
      e = hipMemcpy(r->sph_map, sph_map.data(), sizeof(int2) * sph_map.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_pairs > 0) e = hipMalloc((void**)&r->pairs, sizeof(int2) * n_pairs);
    if (e == hipSuccess && n_pairs > 0) e = hipMalloc((void**)&r->pairs_cc, sizeof(int2) * n_padded);
    if (e == hipSuccess) e = hipMemcpy(r->dev, &h, sizeof h, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(r->spheres, sph.data(), sizeof(float4) * sph.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_pairs > 0)
      e = hipMemcpy(r->pairs, dev_pairs.data(), sizeof(int2) * n_pairs, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_pairs > 0)
      e = hipMemcpy(r->pairs_cc, cc_pairs.data(), sizeof(int2) * n_padded, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      cp_robot_destroy(r);
      return hip_fail(e, "cp_robot_create");
    }
    *out = r;
    return CP_OK;
  } catch (...) {
    return fail(CP_E_ARG, "cp_robot_create: unexpected exception");
  }
}

void cp_robot_destroy(cp_robot* r) {
  if (!r) return;
  rtc_release(r);
  if (r->dev) (void)hipFree(r->dev);
  if (r->spheres) (void)hipFree(r->spheres);
  if (r->pairs) (void)hipFree(r->pairs);
  if (r->pairs_cc) (void)hipFree(r->pairs_cc);
  if (r->sph_map) (void)hipFree(r->sph_map);
  delete r;
}

int cp_robot_self_pairs(const cp_robot* robot, int32_t capacity, int32_t* pairs, int32_t* count) {
  try {
    if (!robot || !count) return fail(CP_E_ARG, "cp_robot_self_pairs: NULL argument");
    if (capacity < 0 || (capacity > 0 && !pairs))
      return fail(CP_E_ARG, "cp_robot_self_pairs: capacity < 0 or NULL pairs");
    const int n = (int)robot->self_pairs.size() / 2;
    *count = n;
    const int copy = std::min(n, capacity);
    if (copy > 0)
      std::memcpy(pairs, robot->self_pairs.data(), sizeof(int32_t) * 2 * (size_t)copy);
    return CP_OK;
  } catch (...) {
    return fail(CP_E_ARG, "cp_robot_self_pairs: unexpected exception");
  }
}

int cp_env_create(const cp_env_desc* d, cp_env** out) {
  try {
    if (!d || !out) return fail(CP_E_ARG, "cp_env_create: NULL argument");
    *out = nullptr;
    const int counts[5] = {d->n_aabb, d->n_obb, d->n_sphere, d->n_capsule, d->n_cylinder};
    const double* src[5] = {d->aabb, d->obb, d->sphere, d->capsule, d->cylinder};
    const int slots[5] = {2, 4, 1, 2, 2};   // float4 per primitive
    size_t total = 0, n_prims = 0;
    for (int t = 0; t < 5; ++t) {
      if (counts[t] < 0) return fail(CP_E_ARG, "negative primitive count");
      if (counts[t] > 0 && !src[t]) return fail(CP_E_ARG, "NULL primitive array with count %d", counts[t]);
      total += (size_t)counts[t] * slots[t];
      n_prims += (size_t)counts[t];
    }
    if (n_prims > 65535) return fail(CP_E_UNSUPPORTED, "%zu primitives (at most 65535)", n_prims);
    // layout: per-type records, then one bounding sphere per primitive
    std::vector<float4> buf(std::max<size_t>(total + n_prims, 1));
    size_t off[5];
    size_t at = 0;
    for (int t = 0; t < 5; ++t) {
      off[t] = at;
      at += (size_t)counts[t] * slots[t];
    }
    const size_t boff = at;
    size_t bi = boff;
    auto bound = [&](double x, double y, double z, double r) {
      // centre and (radius + culling margin)^2; float rounding of the
      // centre is covered by the margin
      const double reach = r * (1.0 + 1e-6) + (double)kCullMargin;
      buf[bi++] = make_float4((float)x, (float)y, (float)z, (float)(reach * reach));
    };
    for (int i = 0; i < d->n_aabb; ++i) {
      const double* p = d->aabb + 6 * i;
      buf[off[0] + 2 * i] = make_float4((float)p[0], (float)p[1], (float)p[2], 0.f);
      buf[off[0] + 2 * i + 1] = make_float4((float)p[3], (float)p[4], (float)p[5], 0.f);
      bound(p[0], p[1], p[2], std::sqrt(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]));
    }
    for (int i = 0; i < d->n_obb; ++i) {
      const double* p = d->obb + 15 * i;
      // box axis c = column c of R; slot 0 holds the centre's coordinate
      // along each axis, so the device projects a point with one dot product
      double oc[3];
      for (int c = 0; c < 3; ++c) {
        oc[c] = p[3 + c] * p[0] + p[6 + c] * p[1] + p[9 + c] * p[2];
        buf[off[1] + 4 * i + 1 + c] = make_float4((float)p[3 + c], (float)p[6 + c], (float)p[9 + c],
                                                  (float)p[12 + c]);
      }
      buf[off[1] + 4 * i] = make_float4((float)oc[0], (float)oc[1], (float)oc[2], 0.f);
      bound(p[0], p[1], p[2], std::sqrt(p[12] * p[12] + p[13] * p[13] + p[14] * p[14]));
    }
    for (int i = 0; i < d->n_sphere; ++i) {
      const double* p = d->sphere + 4 * i;
      buf[off[2] + i] = make_float4((float)p[0], (float)p[1], (float)p[2], (float)p[3]);
      bound(p[0], p[1], p[2], p[3]);
    }
    for (int i = 0; i < d->n_capsule; ++i) {
      const double* p = d->capsule + 7 * i;
      const double dx = p[3] - p[0], dy = p[4] - p[1], dz = p[5] - p[2];
      const double dd = dx * dx + dy * dy + dz * dz;
      buf[off[3] + 2 * i] = make_float4((float)p[0], (float)p[1], (float)p[2], (float)p[6]);
      buf[off[3] + 2 * i + 1] = make_float4((float)dx, (float)dy, (float)dz, dd > 0 ? (float)(1.0 / dd) : 0.f);
      bound(p[0] + 0.5 * dx, p[1] + 0.5 * dy, p[2] + 0.5 * dz, 0.5 * std::sqrt(dd) + p[6]);
    }
    for (int i = 0; i < d->n_cylinder; ++i) {
      const double* p = d->cylinder + 8 * i;
      const double n = std::sqrt(p[3] * p[3] + p[4] * p[4] + p[5] * p[5]);
      if (std::fabs(n - 1.0) > 1e-6) return fail(CP_E_ARG, "cylinder %d: axis is not a unit vector", i);
      buf[off[4] + 2 * i] = make_float4((float)p[0], (float)p[1], (float)p[2], (float)p[6]);
      buf[off[4] + 2 * i + 1] = make_float4((float)p[3], (float)p[4], (float)p[5], (float)p[7]);
      bound(p[0], p[1], p[2], std::sqrt(p[6] * p[6] + p[7] * p[7]));
    }
    cp_env* env = new (std::nothrow) cp_env;
    if (!env) return fail(CP_E_ARG, "out of host memory");
    hipError_t e = hipMalloc((void**)&env->block, sizeof(float4) * buf.size());
    if (e == hipSuccess) e = hipMemcpy(env->block, buf.data(), sizeof(float4) * buf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      cp_env_destroy(env);
      return hip_fail(e, "cp_env_create");
    }
    env->total = (int)n_prims;
    EnvDev& v = env->view;
    v.n_aabb = d->n_aabb; v.n_obb = d->n_obb; v.n_sph = d->n_sphere;
    v.n_cap = d->n_capsule; v.n_cyl = d->n_cylinder;
    v.aabb = env->block + off[0];
    v.obb = env->block + off[1];
    v.sph = env->block + off[2];
    v.cap = env->block + off[3];
    v.cyl = env->block + off[4];
    v.bound = env->block + boff;
    *out = env;
    return CP_OK;
  } catch (...) {
    return fail(CP_E_ARG, "cp_env_create: unexpected exception");
  }
}

void cp_env_destroy(cp_env* env) {
  if (!env) return;
  if (env->block) (void)hipFree(env->block);
  delete env;
}

int fk_cc_batch(const cp_robot* robot, const cp_env* env, int32_t n_cfg, const float* d_q,
                uint8_t* d_collide, float* d_min_sd, float* d_sphere_xyz, int32_t flags,
                void* stream) {
  try {
    if (!robot || !env) return fail(CP_E_ARG, "fk_cc_batch: NULL handle");
    if (n_cfg < 0) return fail(CP_E_ARG, "fk_cc_batch: n_cfg < 0");
    if (n_cfg == 0) return CP_OK;
    if (!d_q || !d_collide) return fail(CP_E_ARG, "fk_cc_batch: NULL buffer");
    const bool early = !(flags & CP_NO_EARLY_EXIT);
    // the kernel compiled for this robot (cp_robot_specialize) for the
    // verdicts alone; the signed distances take the library kernel
    RtcFns rk;
    hipError_t e;
    if (!d_min_sd && !(flags & CP_GENERIC) &&
        rtc_find_validate(const_cast<cp_robot*>(robot), &rk) && rk.fkcc[1]) {
      e = launch_rtc_fk_cc(rk, robot, env->view, n_cfg, d_q, d_collide, early, 8, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "fk_cc_batch launch (run-time compiled kernel)");
    } else {
      e = launch_fk_cc(robot->dev, robot->spheres, env->view, n_cfg, d_q, d_collide, d_min_sd, early,
                       8, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "fk_cc_batch launch");
    }
    if (d_sphere_xyz) {
      e = launch_sphere_xyz(robot->dev, robot->spheres, robot->sph_map, robot->host.n_spheres,
                            n_cfg, d_q, d_sphere_xyz, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "fk_cc_batch sphere centre launch");
    }
    if (flags & CP_SELF_COLLISION) {
      e = launch_self_cc(robot->dev, robot->host, robot->spheres, robot->pairs_cc, robot->n_cc,
                         n_cfg, d_q, d_collide, d_min_sd, early, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "fk_cc_batch self-collision launch");
    }
    return CP_OK;
  } catch (...) {
    return fail(CP_E_ARG, "fk_cc_batch: unexpected exception");
  }
}

namespace {

int check_params(const cp_proj_params* params, cp_proj_params* p) {
  cp_proj_params_default(p);
  if (params) *p = *params;
  if (p->W != 32 && p->W != 64) return fail(CP_E_UNSUPPORTED, "W = %d (supported: 32, 64)", p->W);
  if (p->max_iters < 1) return fail(CP_E_ARG, "max_iters < 1");
  if (!(p->tau >= 0) || !(p->tau_sm >= 0) || !(p->tau_task >= 0) || !(p->lambda >= 0) ||
      !(p->alpha > 0))
    return fail(CP_E_ARG, "projection parameters out of range");
  if (p->sphere_batch != 4 && p->sphere_batch != 8 && p->sphere_batch != 16)
    return fail(CP_E_UNSUPPORTED, "sphere_batch = %d (supported: 4, 8, 16)", p->sphere_batch);
  if (p->variant < CP_PROJECT_PARALLEL || p->variant > CP_PROJECT_SEQUENTIAL)
    return fail(CP_E_ARG, "variant = %d (CP_PROJECT_*)", p->variant);
  return CP_OK;
}

int do_project(const cp_robot* robot, const cp_constraint* constraint, const cp_proj_params& p,
               int32_t n_motions, const float* d_q_from, const float* d_q_to, float* d_xi,
               int32_t* d_status, int32_t* d_iters, uint64_t* d_work, int32_t flags, void* stream) {
  if (!dof_supported(robot->host.dof))
    return fail(CP_E_UNSUPPORTED, "projection kernels are built for dof 2, 3, 6, 7, 9, 14 (got %d)", robot->host.dof);
  ConDev con;
  int rc = make_constraint(constraint, robot, &con);
  if (rc != CP_OK) return rc;
  if (n_motions == 0) return CP_OK;
  if (!d_q_from || !d_q_to || !d_xi || !d_status) return fail(CP_E_ARG, "NULL buffer");
  ProjDev prm;
  prm.W = p.W;
  prm.max_iters = p.max_iters;
  prm.tau = (float)p.tau;
  prm.tau_sm = (float)p.tau_sm;
  prm.tau_task = (float)p.tau_task;
  prm.alpha = (float)p.alpha;
  prm.lambda2 = (float)(p.lambda * p.lambda);
  prm.variant = p.variant;
  if ((flags & CP_POOLED) && (flags & CP_PER_MOTION))
    return fail(CP_E_ARG, "CP_POOLED and CP_PER_MOTION together");
  const int pooled = (flags & CP_POOLED) ? 1 : (flags & CP_PER_MOTION) ? 0 : -1;
  // the kernel compiled for this robot and mask (cp_robot_specialize), when
  // the pooled form is the one to run
  if (!(flags & CP_GENERIC) && p.variant != CP_PROJECT_SEQUENTIAL && use_pool(n_motions, pooled)) {
    RtcFns rk;
    if (rtc_find(const_cast<cp_robot*>(robot), con, &rk) && rk.pool) {
      hipError_t e = launch_rtc_pool(rk, robot, con, prm, n_motions, d_q_from, d_q_to, d_xi,
                                     d_status, d_iters, (unsigned long long*)d_work,
                                     (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "projection launch (run-time compiled kernel)");
      return CP_OK;
    }
  }
  bool supported = false;
  hipError_t e = launch_project(robot->host.dof, robot->dev, con, prm, n_motions, d_q_from, d_q_to,
                                d_xi, d_status, d_iters, (unsigned long long*)d_work, pooled,
                                (hipStream_t)stream, &supported);
  if (!supported) return fail(CP_E_UNSUPPORTED, "no kernel for dof %d with constraint kind %d", robot->host.dof, con.kind);
  if (e != hipSuccess) return hip_fail(e, "projection launch");
  return CP_OK;
}

int do_validate(const cp_robot* robot, const cp_env* env, const cp_proj_params& p,
                int32_t n_motions, const float* d_xi, int32_t* d_status, uint64_t* d_work,
                int32_t flags, void* stream) {
  if (n_motions == 0) return CP_OK;
  if (!d_xi || !d_status) return fail(CP_E_ARG, "NULL buffer");
  // the kernels compiled for this robot (cp_robot_specialize), for the
  // culled form
  RtcFns rk;
  if (!(flags & (CP_GENERIC | CP_NO_CULL)) && rtc_find_validate(const_cast<cp_robot*>(robot), &rk)) {
    hipError_t e = launch_rtc_validate(rk, robot, env->view, p.W, n_motions, d_xi, d_status,
                                       (unsigned long long*)d_work, !(flags & CP_NO_EARLY_EXIT),
                                       p.sphere_batch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "validation launch (run-time compiled kernel)");
  } else {
    hipError_t e = launch_validate(robot->dev, robot->spheres, env->view, p.W, n_motions, d_xi,
                                   d_status, (unsigned long long*)d_work,
                                   !(flags & CP_NO_EARLY_EXIT), !(flags & CP_NO_CULL),
                                   p.sphere_batch, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "validation launch");
  }
  if (flags & CP_SELF_COLLISION) {
    hipError_t e = launch_self_cc_motions(robot->dev, robot->host, robot->spheres, robot->pairs_cc,
                                          robot->n_cc, p.W, n_motions, d_xi, d_status,
                                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "self-collision launch");
  }
  return CP_OK;
}

}  // namespace

int project_motions(const cp_robot* robot, const cp_constraint* constraint,
                    const cp_proj_params* params, int32_t n_motions, const float* d_q_from,
                    const float* d_q_to, float* d_xi, int32_t* d_status, int32_t* d_iters,
                    uint64_t* d_work, void* stream) {
  try {
    if (!robot) return fail(CP_E_ARG, "project_motions: NULL handle");
    if (n_motions < 0) return fail(CP_E_ARG, "project_motions: n_motions < 0");
    cp_proj_params p;
    int rc = check_params(params, &p);
    if (rc != CP_OK) return rc;
    return do_project(robot, constraint, p, n_motions, d_q_from, d_q_to, d_xi, d_status, d_iters,
                      d_work, 0, stream);
  } catch (...) {
    return fail(CP_E_ARG, "project_motions: unexpected exception");
  }
}

int validate_motions(const cp_robot* robot, const cp_env* env, const cp_proj_params* params,
                     int32_t n_motions, const float* d_xi, int32_t* d_status, uint64_t* d_work,
                     int32_t flags, void* stream) {
  try {
    if (!robot || !env) return fail(CP_E_ARG, "validate_motions: NULL handle");
    if (n_motions < 0) return fail(CP_E_ARG, "validate_motions: n_motions < 0");
    cp_proj_params p;
    int rc = check_params(params, &p);
    if (rc != CP_OK) return rc;
    return do_validate(robot, env, p, n_motions, d_xi, d_status, d_work, flags, stream);
  } catch (...) {
    return fail(CP_E_ARG, "validate_motions: unexpected exception");
  }
}

int project_validate_motions(const cp_robot* robot, const cp_env* env,
                             const cp_constraint* constraint, const cp_proj_params* params,
                             int32_t n_motions, const float* d_q_from, const float* d_q_to,
                             float* d_xi, int32_t* d_status, int32_t* d_iters, uint64_t* d_work,
                             int32_t flags, void* stream) {
  try {
    if (!robot || !env) return fail(CP_E_ARG, "project_validate_motions: NULL handle");
    if (n_motions < 0) return fail(CP_E_ARG, "project_validate_motions: n_motions < 0");
    cp_proj_params p;
    int rc = check_params(params, &p);
    if (rc != CP_OK) return rc;
    rc = do_project(robot, constraint, p, n_motions, d_q_from, d_q_to, d_xi, d_status, d_iters,
                    d_work, flags, stream);
    if (rc != CP_OK) return rc;
    return do_validate(robot, env, p, n_motions, d_xi, d_status, d_work, flags, stream);
  } catch (...) {
    return fail(CP_E_ARG, "project_validate_motions: unexpected exception");
  }
}

int project_configs(const cp_robot* robot, const cp_constraint* constraint, int32_t n,
                    const float* d_q_in, float* d_q_out, int32_t* d_status, double tol,
                    int32_t max_iters, double alpha, double lambda, void* stream) {
  try {
    if (!robot) return fail(CP_E_ARG, "project_configs: NULL handle");
    if (n < 0 || max_iters < 0 || !(tol >= 0) || !(alpha > 0) || !(lambda >= 0))
      return fail(CP_E_ARG, "project_configs: argument out of range");
    if (!dof_supported(robot->host.dof))
      return fail(CP_E_UNSUPPORTED, "projection kernels are built for dof 2, 3, 6, 7, 9, 14 (got %d)", robot->host.dof);
    ConDev con;
    int rc = make_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    if (n == 0) return CP_OK;
    if (!d_q_in || !d_q_out || !d_status) return fail(CP_E_ARG, "project_configs: NULL buffer");
    bool supported = false;
    hipError_t e = launch_project_configs(robot->host.dof, robot->dev, con, n, d_q_in, d_q_out,
                                          d_status, (float)tol, max_iters, (float)alpha,
                                          (float)(lambda * lambda), (hipStream_t)stream, &supported);
    if (!supported) return fail(CP_E_UNSUPPORTED, "no kernel for dof %d with constraint kind %d", robot->host.dof, con.kind);
    if (e != hipSuccess) return hip_fail(e, "project_configs launch");
    return CP_OK;
  } catch (...) {
    return fail(CP_E_ARG, "project_configs: unexpected exception");
  }
}

}  // extern "C"

namespace cprrtc {
int api_params(const cp_proj_params* params, cp_proj_params* p) { return check_params(params, p); }
}  // namespace cprrtc
