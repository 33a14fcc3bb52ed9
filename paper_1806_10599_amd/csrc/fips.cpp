// Host set-up and evaluation of the non-local fatigue indicators (see
// fips.hpp).  Band geometry (Sec. 3.3, Eq. 26): the reference point of a
// grain is the centre of its voxel of lowest index; a voxel's offset d from
// it is the periodic minimal image; its coordinate along a slip-plane
// normal n is s = (d0 n0 + d1 n1) + d2 n2 and its band index
// floor(s / w + 1/2).  Every decision is taken in FP64 in this order, with
// no fused multiply-add.
#include "fips.hpp"

#include <cmath>
#include <cstring>

namespace rve {

void FipIndex::ensure(void** p, size_t& cap, size_t bytes, const Alloc& alloc,
                      const Release& release) {
  if (bytes <= cap && *p) return;
  if (*p) release(*p);
  *p = nullptr;
  cap = 0;
  *p = alloc(bytes < 256 ? 256 : bytes);
  cap = bytes < 256 ? 256 : bytes;
}

#pragma clang fp contract(off)
FipLists fip_lists(int n, const double L[3], const int32_t* phase,
                   const double* table, int G, double width) {
  if (!(width > 0.0) || !std::isfinite(width))
    throw Error(RVE_EINVAL, "band width must be finite and > 0");
  FipLists out;
  auto& segs = out.segs;
  auto& grain_label_ = out.grain_label;
  auto& band_meta_ = out.band_meta;
  const int64_t N = (int64_t)n * n * n;
  std::vector<int64_t> first(G, -1), count(G, 0);
  auto crystal = [&](int g) { return table[(size_t)g * kTableStride] == 0.0; };
  for (int64_t v = 0; v < N; ++v) {
    const int g = phase[v];
    if (!crystal(g)) continue;
    if (first[g] < 0) first[g] = v;
    ++count[g];
  }
  // voxel centres along each axis
  std::vector<double> xc[3];
  for (int a = 0; a < 3; ++a) {
    xc[a].resize(n);
    const double h = L[a] / (double)n;
    for (int i = 0; i < n; ++i) xc[a][i] = ((double)i + 0.5) * h;
  }
  // band index of every crystal voxel on every plane
  std::vector<int64_t> jv((size_t)4 * N, 0);
  std::vector<int64_t> jmin((size_t)G * 4, INT64_MAX), jmax((size_t)G * 4, INT64_MIN);
  for (int64_t v = 0; v < N; ++v) {
    const int g = phase[v];
    if (!crystal(g)) continue;
    const int64_t r = first[g];
    const int64_t iv[3] = {v / ((int64_t)n * n), (v / n) % n, v % n};
    const int64_t ir[3] = {r / ((int64_t)n * n), (r / n) % n, r % n};
    double d[3];
    for (int a = 0; a < 3; ++a) {
      double t = xc[a][iv[a]] - xc[a][ir[a]];
      t = t - L[a] * std::floor(t / L[a] + 0.5);
      d[a] = t;
    }
    const double* tab = table + (size_t)g * kTableStride;
    for (int p = 0; p < 4; ++p) {
      const double* m = tab + kTabM + 3 * (3 * p);
      const double s = (d[0] * m[0] + d[1] * m[1]) + d[2] * m[2];
      const double q = std::floor(s / width + 0.5);
      if (!(std::fabs(q) < 1e9)) throw Error(RVE_EINVAL, "band width too small");
      const int64_t j = (int64_t)q;
      jv[(size_t)4 * v + p] = j;
      int64_t& lo = jmin[(size_t)4 * g + p];
      int64_t& hi = jmax[(size_t)4 * g + p];
      if (j < lo) lo = j;
      if (j > hi) hi = j;
    }
  }
  // grain segments (crystal labels with voxels, ascending label), then band
  // segments ordered by (label, plane, j); voxels ascending in each
  std::vector<int64_t> goff(G, -1);
  int64_t off = 0;
  for (int g = 0; g < G; ++g) {
    if (!crystal(g) || count[g] == 0) continue;
    goff[g] = off;
    segs.push_back(FipSeg{off, (int32_t)count[g], g});
    grain_label_.push_back(g);
    off += count[g];
  }
  const int64_t grain_total = off;
  // per (g, p): dense count over [jmin, jmax]
  std::vector<int64_t> cbase((size_t)G * 4, -1);
  int64_t cells = 0;
  for (int g = 0; g < G; ++g)
    for (int p = 0; p < 4; ++p) {
      const size_t k = (size_t)4 * g + p;
      if (jmin[k] > jmax[k]) continue;
      cbase[k] = cells;
      cells += jmax[k] - jmin[k] + 1;
    }
  std::vector<int64_t> ccount(cells, 0), coff(cells, -1);
  for (int64_t v = 0; v < N; ++v) {
    const int g = phase[v];
    if (!crystal(g)) continue;
    for (int p = 0; p < 4; ++p) {
      const size_t k = (size_t)4 * g + p;
      ++ccount[cbase[k] + jv[(size_t)4 * v + p] - jmin[k]];
    }
  }
  for (int g = 0; g < G; ++g)
    for (int p = 0; p < 4; ++p) {
      const size_t k = (size_t)4 * g + p;
      if (cbase[k] < 0) continue;
      for (int64_t j = jmin[k]; j <= jmax[k]; ++j) {
        const int64_t c = cbase[k] + j - jmin[k];
        if (ccount[c] == 0) continue;
        if (ccount[c] > INT32_MAX || j > INT32_MAX || j < INT32_MIN)
          throw Error(RVE_EINVAL, "band too large");
        coff[c] = off;
        segs.push_back(FipSeg{off, (int32_t)ccount[c], 3 * p});
        band_meta_.push_back({g, p, (int32_t)j, (int32_t)ccount[c]});
        off += ccount[c];
      }
    }
  std::vector<int32_t>& vox = out.vox;
  vox.assign(off > 0 ? off : 1, 0);
  std::vector<int64_t> gfill(G, 0);
  std::vector<int64_t> cfill(cells, 0);
  for (int64_t v = 0; v < N; ++v) {
    const int g = phase[v];
    if (!crystal(g)) continue;
    vox[goff[g] + gfill[g]++] = (int32_t)v;
    for (int p = 0; p < 4; ++p) {
      const size_t k = (size_t)4 * g + p;
      const int64_t c = cbase[k] + jv[(size_t)4 * v + p] - jmin[k];
      vox[coff[c] + cfill[c]++] = (int32_t)v;
    }
  }
  (void)grain_total;
  out.entries = off;
  return out;
}
#pragma clang fp contract(on)

void FipIndex::build(int n, const double L[3], const int32_t* phase,
                     const double* table, int G, double width,
                     const Alloc& alloc, const Release& release) {
  built_ = false;
  FipLists fl = fip_lists(n, L, phase, table, G, width);
  grain_label_ = std::move(fl.grain_label);
  band_meta_ = std::move(fl.band_meta);
  const size_t ng = grain_label_.size(), nb = band_meta_.size();
  const auto& vox = fl.vox;
  const auto& segs = fl.segs;
  ensure((void**)&vox_, vox_cap_, vox.size() * sizeof(int32_t), alloc, release);
  ensure((void**)&seg_, seg_cap_, (segs.size() + 1) * sizeof(FipSeg), alloc, release);
  ensure((void**)&res_, res_cap_, (2 * ng + nb + 1) * sizeof(double), alloc, release);
  ensure((void**)&sys_, sys_cap_, (nb + 1) * sizeof(int32_t), alloc, release);
  ensure((void**)&max_, max_cap_, 3 * sizeof(FipMax), alloc, release);
  RVE_HIP(hipMemcpy(vox_, vox.data(), vox.size() * sizeof(int32_t),
                    hipMemcpyHostToDevice));
  if (!segs.empty())
    RVE_HIP(hipMemcpy(seg_, segs.data(), segs.size() * sizeof(FipSeg),
                      hipMemcpyHostToDevice));
  G_ = G;
  width_ = width;
  built_ = true;
}


void FipIndex::evaluate(const double* pcyc, const double* pcyc_lit,
                        const double* w, int64_t cstride, int64_t base,
                        hipStream_t s, rve_nonlocal_fips* out,
                        double* grain_pcyc, double* grain_pcyc_lit,
                        int32_t labels, double* band_wcyc, int32_t* band_desc,
                        int64_t band_cap) {
  if (!built_) throw Error(RVE_ESTATE, "band index not built");
  if (!out) throw Error(RVE_EINVAL, "null summary");
  if ((grain_pcyc || grain_pcyc_lit) && labels != G_)
    throw Error(RVE_EINVAL, "labels must equal the number of microstructure labels");
  const int ng = (int)grain_label_.size();
  const int64_t nb = (int64_t)band_meta_.size();
  launch_fip_grain_means(vox_, seg_, ng, pcyc, pcyc_lit, base, res_, s);
  launch_fip_band_means(vox_, seg_ + ng, (int)nb, w, cstride, base,
                        res_ + 2 * ng, sys_, s);
  if (ng > 0) {
    launch_fip_argmax(res_, ng, max_, s);
    launch_fip_argmax(res_ + ng, ng, max_ + 1, s);
  }
  if (nb > 0) launch_fip_argmax(res_ + 2 * ng, nb, max_ + 2, s);
  RVE_HIP(hipGetLastError());
  FipMax mx[3] = {};
  std::vector<double> res(2 * (size_t)ng + nb);
  std::vector<int32_t> sys(nb);
  RVE_HIP(hipMemcpyAsync(mx, max_, sizeof(mx), hipMemcpyDeviceToHost, s));
  if (!res.empty())
    RVE_HIP(hipMemcpyAsync(res.data(), res_, res.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  if (nb > 0)
    RVE_HIP(hipMemcpyAsync(sys.data(), sys_, nb * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
  RVE_HIP(hipStreamSynchronize(s));
  std::memset(out, 0, sizeof(*out));
  out->band_width = width_;
  out->grains = ng;
  out->bands = nb;
  out->pcyc_label = out->pcyc_lit_label = -1;
  out->wcyc_band = -1;
  out->wcyc_label = out->wcyc_plane = out->wcyc_system = -1;
  if (ng > 0) {
    out->pcyc_g = mx[0].val;
    out->pcyc_label = grain_label_[mx[0].idx];
    out->pcyc_lit_g = mx[1].val;
    out->pcyc_lit_label = grain_label_[mx[1].idx];
  }
  if (nb > 0) {
    const auto& m = band_meta_[mx[2].idx];
    out->wcyc_b = mx[2].val;
    out->wcyc_band = mx[2].idx;
    out->wcyc_label = m[0];
    out->wcyc_plane = m[1];
    out->wcyc_j = m[2];
    out->wcyc_voxels = m[3];
    out->wcyc_system = sys[mx[2].idx];
  }
  if (grain_pcyc || grain_pcyc_lit) {
    for (int g = 0; g < G_; ++g) {
      if (grain_pcyc) grain_pcyc[g] = 0.0;
      if (grain_pcyc_lit) grain_pcyc_lit[g] = 0.0;
    }
    for (int k = 0; k < ng; ++k) {
      if (grain_pcyc) grain_pcyc[grain_label_[k]] = res[k];
      if (grain_pcyc_lit) grain_pcyc_lit[grain_label_[k]] = res[ng + k];
    }
  }
  if (band_wcyc || band_desc) {
    if (band_cap < nb) throw Error(RVE_EINVAL, "band arrays smaller than the band count");
    for (int64_t b = 0; b < nb; ++b) {
      if (band_wcyc) band_wcyc[b] = res[2 * ng + b];
      if (band_desc) {
        const auto& m = band_meta_[b];
        int32_t* d = band_desc + 5 * b;
        d[0] = m[0];
        d[1] = m[1];
        d[2] = m[2];
        d[3] = sys[b];
        d[4] = m[3];
      }
    }
  }
}

}  // namespace rve
