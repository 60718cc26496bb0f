// Patch form of the operator passes: declarations shared by the host set-up
// (patch_setup.cpp), the device set-up (setup.hip) and the kernels (patch.hip).
#pragma once

#include <cstdint>
#include <vector>

namespace bras {

// Host result of the patch partition (patch_setup.cpp).  Element indices in
// pe are internal (patch-major); perm maps them back to the caller's order.
struct PatchPlan {
  int64_t npatch = 0;
  std::vector<int32_t> perm;    // [E] internal element -> caller's element
  std::vector<int32_t> pe;      // [npatch+1] internal elements of each patch
  std::vector<int32_t> pd;      // [npatch+1] range of each patch's DOF list in pdof
  std::vector<int32_t> pnl;     // [npatch] DOFs of the patch whose copies all lie in it (listed first)
  std::vector<int32_t> pdof;    // patch DOF lists (conforming DOF numbers)
  std::vector<uint16_t> code;   // [E*nl] copy (e, l) of patch p at pe[p]*nl + l*ne_p + e: j | rank << lbits
  std::vector<int32_t> sbase;   // [npatch+1] first partial of each patch's shared DOFs (patch-major)
  std::vector<int32_t> srp;     // [ns+1] partials of shared DOF s: spos[srp[s] .. srp[s+1]), in patch order
  std::vector<int32_t> spos;    // partial indices
  std::vector<int32_t> sdof;    // [ns] the shared DOFs, increasing
  // internal DOF numbering of the solvers' vectors: the local DOFs of patch 0,
  // of patch 1, ..., then the shared DOFs in sdof order
  std::vector<int32_t> ip2g;    // [n] internal -> conforming DOF
  std::vector<int32_t> pidx;    // like pdof, internal numbers
  int64_t nloc_total = 0;       // DOFs local to some patch (the first internal numbers)
  int lbits = 0, rbits = 0, maxrank = 0, maxdofs = 0;
};

// Partition (at most P elements and Dmax DOFs per patch) and patch maps for
// the map l2g [E][nl] with multiplicities mult [n].  Codes are 16-bit, so the
// DOF cap is lowered until j and rank fit (rank < max multiplicity).  Returns
// 0 on success, 1 when no plan fits (the operator passes then keep the
// element / reduce form).
int build_patch_plan(int64_t n, int64_t E, int nl, const int32_t* l2g, const int32_t* mult, int P, int Dmax,
                     PatchPlan* plan);

// Device copy of the plan (owned by the handle).
struct PatchDev {
  int64_t npatch = 0;
  int64_t ns = 0;          // shared DOFs
  int64_t nspart = 0;      // partial sums of shared DOFs
  int lbits = 0, maxrank = 0, maxdofs = 0;
  int maxelems = 0;        // elements of the largest patch
  int nb2 = 0;             // work-groups of the shared-DOF pass
  int32_t* perm = nullptr;
  int32_t* pe = nullptr;
  int32_t* pd = nullptr;
  int32_t* pnl = nullptr;
  int32_t* pdof = nullptr;
  uint16_t* code = nullptr;
  int32_t* sbase = nullptr;
  int32_t* srp = nullptr;
  int32_t* spos = nullptr;
  int32_t* sdof = nullptr;
  double* part = nullptr;  // [nspart] partial sums (the handle's workspace)
  // internal DOF numbering (the solvers' vectors while a patch-form solve runs)
  int64_t nloc_total = 0;
  int32_t* ip2g = nullptr;
  int32_t* pidx = nullptr;
  double* invd_ip = nullptr;      // D^-1 in internal numbering
  double* invdiag_ip = nullptr;   // diag(M)^-1 in internal numbering
};

// Work-group size of the patch pass: at most this many elements per patch.
constexpr int kPatchBlock = 256;
// Default patch size and DOF cap (LDS holds one float64 per patch DOF).
constexpr int kPatchElems = 256;
constexpr int kPatchMaxDofs = 3072;
// Shared-DOF pass: each thread sums kPatchSharedPerThread shared DOFs
// (independent loads in flight), so a work-group covers kPatchSharedPerBlock.
constexpr int kPatchSharedPerThread = 2;
constexpr int kPatchSharedPerBlock = kPatchBlock * kPatchSharedPerThread;
constexpr int kPatchSharedBlocks = 1 << 20;

}  // namespace bras
