// Non-local fatigue indicators (Sec. 3.3, Eqs. 25-26): grain averages of
// P_cyc and slip-band averages of W_cyc^a, and their maxima over the RVE.
//
// Set-up (host, once per microstructure and band width): the voxels of
// every crystal grain in ascending index order, and for each grain and
// each of its four {111} slip planes the voxels of every band of the
// requested width, grouped band by band.  Evaluation (device, at any
// time): one wavefront per grain or band sums its voxels in a fixed order,
// then a one-block kernel takes the maxima (first index among equal
// values), so the results are bitwise reproducible.
#pragma once

#include <array>
#include <functional>
#include <vector>

#include "../../include/rve.h"
#include "kernels.hpp"

namespace rve {

// one grain or band: voxels vox[off, off + len); comp = first W component
// of the band's plane (3 p) for bands
struct FipSeg {
  int64_t off;
  int32_t len;
  int32_t comp;
};

struct FipMax {
  double val;
  int32_t idx;
  int32_t pad;
};

void launch_fip_grain_means(const int32_t* vox, const FipSeg* seg, int nseg,
                            const double* pcyc, const double* pcyc_lit,
                            int64_t base, double* out, hipStream_t s);
void launch_fip_band_means(const int32_t* vox, const FipSeg* seg, int nseg,
                           const double* w, int64_t cstride, int64_t base,
                           double* val, int32_t* sys, hipStream_t s);
void launch_fip_argmax(const double* v, int64_t n, FipMax* out, hipStream_t s);

// host band lists (no device work): grain segments (ascending label), then
// band segments in (label, plane, j) order, offsets into vox; vox holds the
// voxel indices of every segment, ascending within a segment
struct FipLists {
  std::vector<FipSeg> segs;
  std::vector<int32_t> vox;
  std::vector<int32_t> grain_label;                  // per grain segment
  std::vector<std::array<int32_t, 4>> band_meta;     // label, plane, j, len
  int64_t entries = 0;                               // used entries of vox
};
FipLists fip_lists(int n, const double L[3], const int32_t* phase,
                   const double* table, int G, double width);

class FipIndex {
 public:
  using Alloc = std::function<void*(size_t)>;
  using Release = std::function<void(void*)>;

  // n: grid edge; L: cell lengths; phase: host [n^3] labels; table: host
  // label tables [G][kTableStride] (law at 0, sample-frame normals at
  // kTabM); width > 0
  void build(int n, const double L[3], const int32_t* phase,
             const double* table, int G, double width, const Alloc& alloc,
             const Release& release);
  bool built_for(double width) const { return built_ && width == width_; }
  void invalidate() { built_ = false; }

  // evaluates on the device and fills *out (and the optional host arrays)
  void evaluate(const double* pcyc, const double* pcyc_lit, const double* w,
                int64_t cstride, int64_t base, hipStream_t s,
                rve_nonlocal_fips* out, double* grain_pcyc,
                double* grain_pcyc_lit, int32_t labels, double* band_wcyc,
                int32_t* band_desc, int64_t band_cap);

 private:
  void ensure(void** p, size_t& cap, size_t bytes, const Alloc& alloc,
              const Release& release);

  bool built_ = false;
  double width_ = 0.0;
  int G_ = 0;
  // host metadata
  std::vector<int32_t> grain_label_;                 // per grain segment
  std::vector<std::array<int32_t, 4>> band_meta_;    // label, plane, j, len
  // device
  int32_t* vox_ = nullptr;
  size_t vox_cap_ = 0;
  FipSeg* seg_ = nullptr;     // grain segments, then band segments
  size_t seg_cap_ = 0;
  double* res_ = nullptr;     // grain means [2][ng], band values [nb]
  size_t res_cap_ = 0;
  int32_t* sys_ = nullptr;    // band systems [nb]
  size_t sys_cap_ = 0;
  FipMax* max_ = nullptr;     // 3 results
  size_t max_cap_ = 0;
};

}  // namespace rve
