// Host construction of the projector tables.
//
// The non-local terms of H~ and S~ (Eq. (dh) and the overlap operator beside
// it) need the grid values of every projector p~^a_i. For a Bloch system the
// value at grid point r of the cell is q^a_i(r) = sum_R exp(i k.R) p~^a_i(r - R_a - R)
// over all lattice vectors R that bring the sphere of radius rc onto r.
// We enumerate the unwrapped grid points inside each atom's sphere, fold them
// into the cell (this fold fixes R), evaluate the projector there and sum
// duplicates (a sphere larger than the cell meets its own images).
//
// Projector shape (synthetic stand-in for setup data): channel (l, sigma, rc)
// has 2l+1 functions N r^l exp(-r^2/2sigma^2) (1-(r/rc)^2)^2 Y_lm, with
// N = [Gamma(l+3/2) sigma^(2l+3)/2]^(-1/2) and real harmonics in the order
// m = -l..l: (y, z, x) for l = 1, (xy, yz, 3z^2-r^2, xz, x^2-y^2) for l = 2.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace gfd {

namespace {

constexpr double kPi = 3.14159265358979323846;

int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// All ni projector values at displacement (x, y, z) from the atom.
void projector_values(const gpaw_channel *ch, int nchan, double x, double y, double z,
                      double *out) {
  const double r2 = x * x + y * y + z * z;
  const double r = std::sqrt(r2);
  int i = 0;
  for (int c = 0; c < nchan; ++c) {
    const int l = ch[c].l;
    const double sg = ch[c].sigma, rc = ch[c].rc;
    const double s = r / rc;
    const double chi = s < 1.0 ? (1.0 - s * s) * (1.0 - s * s) : 0.0;
    const double norm = 1.0 / std::sqrt(std::tgamma(l + 1.5) * std::pow(sg, 2 * l + 3) * 0.5);
    const double rad = norm * std::exp(-r2 / (2.0 * sg * sg)) * chi;
    if (l == 0) {
      out[i++] = rad * 0.5 / std::sqrt(kPi);
    } else if (l == 1) {
      const double c1 = std::sqrt(3.0 / (4.0 * kPi));
      out[i++] = rad * c1 * y;
      out[i++] = rad * c1 * z;
      out[i++] = rad * c1 * x;
    } else {
      const double c2 = 0.5 * std::sqrt(15.0 / kPi);
      const double c20 = 0.25 * std::sqrt(5.0 / kPi);
      const double c22 = 0.25 * std::sqrt(15.0 / kPi);
      out[i++] = rad * c2 * x * y;
      out[i++] = rad * c2 * y * z;
      out[i++] = rad * c20 * (3.0 * z * z - r2);
      out[i++] = rad * c2 * x * z;
      out[i++] = rad * c22 * (x * x - y * y);
    }
  }
}

struct Entry {
  int32_t g;
  int32_t atom;
  int64_t slot;  // offset of this entry's ni values in the value pool
};

template <typename T>
int upload(T **dst, const std::vector<T> &src) {
  *dst = nullptr;
  if (src.empty()) return GPAW_OK;
  GFD_HIP(hipMalloc(reinterpret_cast<void **>(dst), src.size() * sizeof(T)));
  GFD_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return GPAW_OK;
}

}  // namespace

int build_tables(const gpaw_sys_desc *d, gpaw_sys *s) {
  const int ni = s->ni;
  const bool cplx = s->dtype == GPAW_C128;
  const int64_t n0 = d->n[0], n1 = d->n[1], n2 = d->n[2];
  double rmax = 0.0;
  for (int c = 0; c < d->nchan; ++c) rmax = std::max(rmax, d->chan[c].rc);

  std::vector<Entry> ent;        // atom-major, sorted by g within an atom
  std::vector<double> pool_re, pool_im;
  std::vector<int32_t> a_start(d->natoms + 1, 0);
  std::vector<double> vals(ni);

  for (int a = 0; a < d->natoms; ++a) {
    a_start[a] = static_cast<int32_t>(ent.size());
    const double *R = d->pos + 3 * a;
    int64_t lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
      lo[c] = static_cast<int64_t>(std::ceil((R[c] - rmax) / d->h[c]));
      hi[c] = static_cast<int64_t>(std::floor((R[c] + rmax) / d->h[c]));
    }
    // (g, phase-weighted values) of every unwrapped point in the sphere
    struct Raw { int32_t g; double re[32]; double im[32]; };
    std::vector<Raw> raw;
    for (int64_t i = lo[0]; i <= hi[0]; ++i) {
      const double dx = i * d->h[0] - R[0];
      for (int64_t j = lo[1]; j <= hi[1]; ++j) {
        const double dy = j * d->h[1] - R[1];
        for (int64_t l = lo[2]; l <= hi[2]; ++l) {
          const double dz = l * d->h[2] - R[2];
          if (dx * dx + dy * dy + dz * dz >= rmax * rmax) continue;
          const int64_t wi = floor_div(i, n0), wj = floor_div(j, n1), wl = floor_div(l, n2);
          const int64_t g = ((i - wi * n0) * n1 + (j - wj * n1)) * n2 + (l - wl * n2);
          projector_values(d->chan, d->nchan, dx, dy, dz, vals.data());
          // unwrapped point = cell point + w L, i.e. image R = -w L: phase exp(-2 pi i k.w)
          const double arg = -2.0 * kPi * (d->k[0] * wi + d->k[1] * wj + d->k[2] * wl);
          const double cr = cplx ? std::cos(arg) : 1.0, sr = cplx ? std::sin(arg) : 0.0;
          Raw r;
          r.g = static_cast<int32_t>(g);
          for (int q = 0; q < ni; ++q) {
            r.re[q] = cr * vals[q];
            r.im[q] = sr * vals[q];
          }
          raw.push_back(r);
        }
      }
    }
    std::stable_sort(raw.begin(), raw.end(), [](const Raw &x, const Raw &y) { return x.g < y.g; });
    for (size_t p = 0; p < raw.size();) {
      size_t q = p + 1;
      Entry e{raw[p].g, a, static_cast<int64_t>(pool_re.size())};
      double re[32], im[32];
      for (int t = 0; t < ni; ++t) { re[t] = raw[p].re[t]; im[t] = raw[p].im[t]; }
      while (q < raw.size() && raw[q].g == raw[p].g) {
        for (int t = 0; t < ni; ++t) { re[t] += raw[q].re[t]; im[t] += raw[q].im[t]; }
        ++q;
      }
      for (int t = 0; t < ni; ++t) { pool_re.push_back(re[t]); pool_im.push_back(im[t]); }
      ent.push_back(e);
      p = q;
    }
  }
  a_start[d->natoms] = static_cast<int32_t>(ent.size());
  const int64_t nent = static_cast<int64_t>(ent.size());
  if (nent >= (int64_t(1) << 31) / std::max(ni, 1))
    return fail(GPAW_EINVAL, "projector tables too large for 32-bit indexing");

  // atom-major arrays
  std::vector<int32_t> e_g(nent);
  std::vector<double> qa(cplx ? 2 * ni * nent : ni * nent);
  for (int64_t e = 0; e < nent; ++e) {
    e_g[e] = ent[e].g;
    for (int t = 0; t < ni; ++t) {
      const double re = pool_re[ent[e].slot + t], im = pool_im[ent[e].slot + t];
      if (cplx) { qa[2 * (t * nent + e)] = re; qa[2 * (t * nent + e) + 1] = im; }
      else qa[t * nent + e] = re;
    }
  }
  // point-major order: by grid point, then atom
  std::vector<int64_t> order(nent);
  for (int64_t e = 0; e < nent; ++e) order[e] = e;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return ent[x].g != ent[y].g ? ent[x].g < ent[y].g : ent[x].atom < ent[y].atom;
  });
  std::vector<int32_t> g2u(s->ng, -1), u_start, pm_atom(nent);
  std::vector<double> qp(qa.size());
  for (int64_t p = 0; p < nent; ++p) {
    const Entry &e = ent[order[p]];
    if (p == 0 || ent[order[p - 1]].g != e.g) {
      g2u[e.g] = static_cast<int32_t>(u_start.size());
      u_start.push_back(static_cast<int32_t>(p));
    }
    pm_atom[p] = e.atom;
    for (int t = 0; t < ni; ++t) {
      const double re = pool_re[e.slot + t], im = pool_im[e.slot + t];
      if (cplx) { qp[2 * (t * nent + p)] = re; qp[2 * (t * nent + p) + 1] = im; }
      else qp[t * nent + p] = re;
    }
  }
  const int64_t nu = static_cast<int64_t>(u_start.size());
  u_start.push_back(static_cast<int32_t>(nent));

  s->tab.nent = nent;
  s->tab.nu = nu;
  int rc;
  if ((rc = upload(&s->tab.a_start, a_start)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.e_g, e_g)) != GPAW_OK) return rc;
  if ((rc = upload(reinterpret_cast<double **>(&s->tab.e_q), qa)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.g2u, g2u)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.u_start, u_start)) != GPAW_OK) return rc;
  if ((rc = upload(&s->tab.pm_atom, pm_atom)) != GPAW_OK) return rc;
  if ((rc = upload(reinterpret_cast<double **>(&s->tab.pm_q), qp)) != GPAW_OK) return rc;
  return GPAW_OK;
}

}  // namespace gfd
