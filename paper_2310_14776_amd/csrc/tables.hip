// Host construction of the projector geometry.
//
// The non-local terms of H~ and S~ (Eq. (dh) and the overlap operator beside
// it) need the grid values of every projector p~^a_i. For a Bloch system the
// value at grid point r of the cell is q^a_i(r) = sum_R exp(i k.R) p~^a_i(r - R_a - R)
// over the lattice vectors R that bring the sphere of radius rc onto r. Here
// we only enumerate the unwrapped grid points inside each atom's sphere and
// fold each into the cell; the fold fixes R = -w L (w = whole cells crossed).
// Each (point, atom, image) triple is one entry; the kernels evaluate the
// projector values of an entry when they need them (proj.h), and entries of
// one point (several atoms, or one atom's own images in a small cell) are
// summed there.
#include <algorithm>
#include <cmath>
#include <vector>

#include "proj.h"

namespace gfd {

namespace {

constexpr double kPi = 3.14159265358979323846;

int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

struct Entry {
  int32_t g;      // folded grid index
  int32_t atom;
  int16_t u[3];   // unwrapped grid indices
  int8_t w[3];    // cells crossed per axis
};

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
  *dst = nullptr;
  if (src.empty()) return GPAW_OK;
  GFD_HIP(hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)));
  GFD_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return GPAW_OK;
}

int setup_proj(const gpaw_sys_desc *d, ProjDev &P) {
  P = ProjDev{};
  if (d->nchan > PROJ_MAX_CHAN) return fail(GPAW_EINVAL, "at most 8 projector channels");
  P.nchan = d->nchan;
  int i = 0;
  for (int c = 0; c < d->nchan; ++c) {
    const gpaw_channel &ch = d->chan[c];
    P.l[c] = ch.l;
    P.norm[c] = 1.0 / std::sqrt(std::tgamma(ch.l + 1.5) * std::pow(ch.sigma, 2 * ch.l + 3) * 0.5);
    P.rc2inv[c] = 1.0 / (ch.rc * ch.rc);
    P.a2[c] = 1.0 / (2.0 * ch.sigma * ch.sigma);
    const int first_slot = ch.l == 0 ? 0 : (ch.l == 1 ? 1 : 4);
    for (int m = 0; m < 2 * ch.l + 1; ++m) {
      P.ch[i] = static_cast<signed char>(c);
      P.ym[i] = static_cast<signed char>(first_slot + m);
      ++i;
    }
  }
  P.ni = i;
  for (int c = 0; c < d->nchan; ++c) {
    P.same_sigma[c] = -1;
    if (c >= 2 && d->chan[c].sigma == d->chan[0].sigma) P.same_sigma[c] = 0;
    else if (c >= 2 && d->chan[c].sigma == d->chan[1].sigma) P.same_sigma[c] = 1;
  }
  // straight-line layout: l = (0, 0, 1, 1, 2) and the last three channels
  // reuse the Gaussian of channel 0 or 1 (two exponentials per point)
  P.std13 = (d->nchan == 5 && P.l[0] == 0 && P.l[1] == 0 && P.l[2] == 1 && P.l[3] == 1 &&
             P.l[4] == 2 && P.same_sigma[2] >= 0 && P.same_sigma[3] >= 0 &&
             P.same_sigma[4] >= 0) ? 1 : 0;
  for (int c = 0; c < 3; ++c) {
    P.n[c] = d->n[c];
    P.h[c] = d->h[c];
    for (int w = -8; w <= 7; ++w) {
      const double arg = -2.0 * kPi * d->k[c] * w;
      P.ph[c][w + 8] = zmake(std::cos(arg), std::sin(arg));
    }
  }
  return GPAW_OK;
}

}  // namespace

int build_tables_host(const gpaw_sys_desc *d, gpaw_sys *s, HostTables &ht) {
  int rc = setup_proj(d, s->proj);
  if (rc != GPAW_OK) return rc;
  const int64_t n[3] = {d->n[0], d->n[1], d->n[2]};
  double rmax = 0.0;
  for (int c = 0; c < d->nchan; ++c) rmax = std::max(rmax, d->chan[c].rc);

  std::vector<Entry> ent;
  for (int a = 0; a < d->natoms; ++a) {
    const double *R = d->pos + 3 * a;
    int64_t lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
      lo[c] = static_cast<int64_t>(std::ceil((R[c] - rmax) / d->h[c]));
      hi[c] = static_cast<int64_t>(std::floor((R[c] + rmax) / d->h[c]));
    }
    for (int64_t i = lo[0]; i <= hi[0]; ++i) {
      const double dx = i * d->h[0] - R[0];
      for (int64_t j = lo[1]; j <= hi[1]; ++j) {
        const double dy = j * d->h[1] - R[1];
        for (int64_t l = lo[2]; l <= hi[2]; ++l) {
          const double dz = l * d->h[2] - R[2];
          if (dx * dx + dy * dy + dz * dz >= rmax * rmax) continue;
          const int64_t u[3] = {i, j, l};
          // a finite system has no images: points outside the grid carry
          // no projector values
          if (d->boundary == 1 &&
              (i < 0 || i >= n[0] || j < 0 || j >= n[1] || l < 0 || l >= n[2]))
            continue;
          Entry e;
          int64_t f[3];
          for (int c = 0; c < 3; ++c) {
            const int64_t w = floor_div(u[c], n[c]);
            if (w < -8 || w > 7 || u[c] < -32768 || u[c] > 32767)
              return fail(GPAW_EINVAL, "projector spheres reach too many cells away; "
                                       "grow the cell or shrink rc");
            f[c] = u[c] - w * n[c];
            e.u[c] = static_cast<int16_t>(u[c]);
            e.w[c] = static_cast<int8_t>(w);
          }
          e.g = static_cast<int32_t>((f[0] * n[1] + f[1]) * n[2] + f[2]);
          e.atom = a;
          ent.push_back(e);
        }
      }
    }
  }
  const int64_t nent = static_cast<int64_t>(ent.size());
  if (nent >= (int64_t(1) << 31) - 1)
    return fail(GPAW_EINVAL, "projector geometry too large for 32-bit indexing");
  if (d->natoms >= (1 << 19)) return fail(GPAW_EINVAL, "too many atoms");

  // atom-major (already grouped by atom); sort by grid index inside an atom
  std::vector<int32_t> a_start(d->natoms + 1, 0);
  std::stable_sort(ent.begin(), ent.end(), [](const Entry &x, const Entry &y) {
    return x.atom != y.atom ? x.atom < y.atom : x.g < y.g;
  });
  for (int64_t e = 0, a = 0; a <= d->natoms; ++a) {
    while (e < nent && ent[e].atom < a) ++e;
    a_start[a] = static_cast<int32_t>(e);
  }
  std::vector<int32_t> e_g(nent);
  std::vector<short4> e_xyz(nent);
  for (int64_t e = 0; e < nent; ++e) {
    e_g[e] = ent[e].g;
    const Entry &x = ent[e];
    const int code = ((x.w[0] + 8) << 8) | ((x.w[1] + 8) << 4) | (x.w[2] + 8);
    e_xyz[e] = make_short4(x.u[0], x.u[1], x.u[2], static_cast<short>(code));
  }
  // point-major: by grid point, then atom, then image
  std::stable_sort(ent.begin(), ent.end(), [](const Entry &x, const Entry &y) {
    if (x.g != y.g) return x.g < y.g;
    if (x.atom != y.atom) return x.atom < y.atom;
    if (x.w[0] != y.w[0]) return x.w[0] < y.w[0];
    if (x.w[1] != y.w[1]) return x.w[1] < y.w[1];
    return x.w[2] < y.w[2];
  });
  if (nent >= (int64_t(1) << 24)) return fail(GPAW_EINVAL, "more than 2^24 projector entries");
  // per point: the first three entry codes inline (most points have at most
  // three), the count and the index of the first entry in pm_code
  std::vector<int32_t> pm_code(nent);
  std::vector<int4> pinfo(s->ng, make_int4(0, 0, 0, 0));
  std::vector<int32_t> cov;
  int64_t ncov = 0;
  for (int64_t e = 0; e < nent; ++e) {
    const Entry &x = ent[e];
    pm_code[e] = pack_code(x.atom, x.w[0], x.w[1], x.w[2]);
    int4 &pi = pinfo[x.g];
    if (e == 0 || ent[e - 1].g != x.g) {
      ++ncov;
      cov.push_back(static_cast<int32_t>(x.g));
      pi = make_int4(pm_code[e], 0, 0, static_cast<int>(e));
    }
    // the count lives in the top byte: unsigned arithmetic, so counts of
    // 128..255 survive the round trip and 256 is caught
    const unsigned cnt = (static_cast<unsigned>(pi.w) >> 24) + 1u;
    if (cnt > 255u) return fail(GPAW_EINVAL, "more than 255 projector entries at one grid point");
    if (cnt == 2u) pi.y = pm_code[e];
    if (cnt == 3u) pi.z = pm_code[e];
    pi.w = static_cast<int>((cnt << 24) | (static_cast<unsigned>(pi.w) & 0xFFFFFFu));
  }

  s->tab.nent = nent;
  s->tab.ncov = ncov;
  ht.a_start = std::move(a_start);
  ht.e_g = std::move(e_g);
  ht.e_xyz = std::move(e_xyz);
  ht.pinfo = std::move(pinfo);
  ht.pm_code = std::move(pm_code);
  ht.cov = std::move(cov);
  ht.pos.assign(d->pos, d->pos + 3 * d->natoms);
  return GPAW_OK;
}

int upload_tables(gpaw_sys *s, const HostTables &ht) {
  int rc;
  if ((rc = upload(&s->tab.a_start, ht.a_start)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.e_g, ht.e_g)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.e_xyz, ht.e_xyz)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.pinfo, ht.pinfo)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.pm_code, ht.pm_code)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.cov, ht.cov)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.pos, ht.pos)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.proj, std::vector<ProjDev>(1, s->proj))) != GPAW_OK) return rc;
  return GPAW_OK;
}

}  // namespace gfd
