// Internal declarations shared by the kernel translation units and the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ptlm {

// Which per-pixel operation a tile kernel performs between the transforms.
enum TileOp : int {
  OP_FORWARD = 0,  // gather psi, F, write zeta
  OP_LOSS = 1,     // gather psi, F, metric sum (+ optional residual ell')
  OP_LINEARIZE = 2,// gather psi, F, metric, store weighted phasors, F^H(ell' e), overlap-add
  OP_JVP = 3,      // gather d psi, F, Re(conj(e) .)
  OP_VJP = 4,      // w e, F^H, overlap-add
  OP_GGNV = 5,     // gather d psi, F, Re(conj(a) .) a, F^H, overlap-add
  OP_DIAG_EXACT = 6,// conj(a)^2, F, read at 2m', overlap-add of the exact diagonal terms
  OP_VJP_RAND = 7  // r a for a generated sign field r, F^H, overlap-add (stochastic diagonal)
};

// Geometry and buffers of one problem as the kernels see them.
struct Geometry {
  int ny, nx, my, mx, K;
  int metric;  // 0 Gauss, 1 Poisson
  int ggn;     // 0 magnitude-based GGN weight ell''(zeta), 1 intensity-based 4 zeta^2 L''(zeta^2)
  int joint;   // 1: probe part is computed
  float background;
  int nseg;    // number of position segments (= grid * tiles per workgroup)
  int grid;    // workgroups of the tile kernels
  int xform;   // transform of the GGN-vector product: 0 FFT tile kernel, 1 DFT as matrix products,
               // 2 FFT tile kernel with the wide grouping (twice the tiles per workgroup)
  // constant tables in the workspace
  const float2* tw;       // twiddles W_L^(n k), n < L/16, k < 16: L = 32, 64, 128, 256, 48, 96
                          // (offsets 0, 32, 96, 224, 480, 528)
  const int2* pos;        // K (row, col)
  const int* seg_start;   // nseg + 1
  const int4* seg_box;    // nseg: (row0, col0, rows, cols) of the segment's strip
  const long long* seg_off;  // nseg: offset of the strip in `strips` (complex elements)
  const int* otile_ptr;   // object 16x16 tiles -> segments whose strip meets the tile (CSR)
  const int* otile_seg;
  const int* ptile_ptr;   // object 16x16 tiles -> positions whose window meets the tile (CSR)
  const int* ptile_pos;
  int otiles_y, otiles_x;
  // linearisation state
  float2* O_lin;          // N
  float2* P_lin;          // M
  float2* afield;         // K*M: sqrt(ell'') e / sqrt(M), detector order
  float* w2;              // K*M: sqrt of the GGN weight (Poisson or intensity-based GGN, else null)
  double* trace;          // K: sum_m ell''_km
  // scratch
  float2* strips;         // per-segment private overlap-add strips (rewritten by every scatter)
  float2* probe_part;     // nseg * M per-segment probe partial sums
  double* partials;       // grid * 4 per-workgroup FP64 partial sums
  float2* scratch;        // grid * M transform tiles (256 x 256 probes only, else null)
};

struct TileArgs {
  const float2* O;        // object used for the gather / probe products
  const float2* P;        // probe
  const float2* vO;       // direction (GGNV / JVP)
  const float2* vP;       // probe direction (joint), may be null
  const float* y;         // data (LOSS / LINEARIZE)
  const float* win;       // K*M real input (VJP)
  float* rout;            // K*M real output (FORWARD zeta, LOSS residual, JVP)
  const int* predicate;   // if non-null and *predicate == 0 the launch does nothing
  const double* bg_add;   // if non-null, added to the background (surrogate metric, App. E)
  // OP_VJP_RAND: sign field of draw rdraw + (*rdraw_t) * rdraw_mul (rdraw_t nullable) from
  // SplitMix64 seeded with rseed
  unsigned long long rseed;
  unsigned long long rdraw;
  const int* rdraw_t;
  int rdraw_mul;
};

// One problem's part of a batched launch: its geometry, its arguments and the first block
// of the launch that belongs to it.  Blocks are dealt out in runs of whole multiples of 8
// (one per XCD), so a problem's local block index has the XCD of the global one.
struct TileJob {
  Geometry g;
  TileArgs a;
  int block0;
  int nblk;
};

// One problem's part of a batched reduction / diagonal launch.  For the object-side kernels a
// job has otiles_x * otiles_y blocks, for the probe-side ones ceil(M / 64), for the partial
// sums one.  The diagonal kernels write their (Re, Im) weights to outO / outP as floats.
struct RedJob {
  Geometry g;
  float2 *outO, *outP;
  const float2 *vO, *vP;
  const float *dO, *dP;
  const double* lam_dev;  // damping read from the device (null: none)
  const int* pred;        // skip when *pred == 0
  double* sums;           // partial-sum output (sum kernels)
  double* pap;            // nullable: per-block parts of p.Ap, p = v (pair reduction of a PCG product)
  const int* pap_block;   // nullable: the alternating update's active block (0 object, 1 probe)
  int pap_base;           // index of the job's first object block among its p.Ap parts
  int block0;
  int nblk;
  int block1;  // first block of the job in a second launch (probe reduction pass one)
};

// one copy of a multi-copy launch (launch_copies): dst[i] = src[i], i < n, unless *pred == 0
struct CopyItem {
  const float2* src;
  float2* dst;
  size_t n;
  const int* pred;
};
constexpr int MAX_COPIES = 4;

struct CopyJob {
  const float2* src;
  float2* dst;
  size_t n;
  const int* pred;
  int block0;
  int nblk;
};

// tile kernels (kernels_tile.hip)
hipError_t launch_tile(const Geometry& g, int op, const TileArgs& a, hipStream_t s);
// Batched launch over jobs of one probe shape: block b runs job job_of_block[b].
hipError_t launch_tile_batch(int my, int mx, int op, const TileJob* jobs, const int* job_of_block, int nblocks,
                             hipStream_t s);
bool tile_shape_supported(int my, int mx);
int tile_threads(int my, int mx);       // threads per workgroup
int tile_per_wg(int my, int mx);        // tiles (concurrent positions) per workgroup
size_t tile_lds_bytes(int my, int mx);
// 256 x 256 tiles (kernels_tile256.hip): three-stage transform through Geometry::scratch
hipError_t launch_tile256(const Geometry& g, int op, const TileArgs& a, hipStream_t s);
hipError_t launch_tile256_batch(int op, const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s);
size_t tile256_lds_bytes();
// 128 x 128 tiles (kernels_tile128.hip): every op but the exact diagonal (which stays on the
// generic kernel); 512-thread workgroups
bool tile128_handles(int op);
hipError_t launch_tile128(const Geometry& g, int op, const TileArgs& a, hipStream_t s);
hipError_t launch_tile128_batch(int op, const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s);
size_t tile128_lds_bytes();
int tile128_threads();
// FP64 refinement of the stored phasors, sqrt-weights and traces at the pixels of extreme GGN
// weight (kernels_refine.hip); runs after a linearisation with the same geometry and arguments;
// nothing to do (and no launch) when the geometry keeps no sqrt-weights (Gaussian magnitude GGN)
hipError_t launch_refine(const Geometry& g, const TileArgs& a, hipStream_t s);
// DFT-as-MFMA GGN-vector kernel for 16 x 16 and 32 x 32 probes (kernels_dft_mfma.hip), same
// scratch as the tile kernels
bool ggnv_mfma_supported(int my, int mx);
// the transform a new handle starts with: the matrix products for 16 x 16 probes and the wide
// grouping for 32 x 32 (each measured fastest there), the FFT tile kernels otherwise
int default_xform(int my, int mx);
// the wide grouping of the generic FFT tile kernel's GGN-vector product (kernels_tile.hip): for
// probes of at most 4096 pixels on that kernel, workgroups of twice the tiles over the same
// segments, ceil(grid / 2) of them (single problems only: batches keep the standard grouping,
// which gives the same bits)
bool ggnv_wide_supported(int my, int mx);
hipError_t launch_ggnv_mfma(const Geometry& g, const TileArgs& a, hipStream_t s);
// batched form over the tile kernels' block table of a 16 x 16 class (16 segments per block)
hipError_t launch_ggnv_mfma_batch(const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s);
// 48 x 48 and 96 x 96 tiles (kernels_tile3.hip): radix 16 x 3 and 16 x 6 transforms
hipError_t launch_tile3(const Geometry& g, int op, const TileArgs& a, hipStream_t s);
hipError_t launch_tile3_batch(int L, int op, const TileJob* jobs, const int* job_of_block, int nblocks, hipStream_t s);
size_t tile3_lds_bytes(int L);
int tile3_per_wg(int L);

// reductions and vector kernels (kernels_vec.hip)
// out_O = sum of the segment strips [+ lam * dO .* vO]
// lam_dev (nullable) overrides lam with a device scalar.
hipError_t launch_obj_reduce(const Geometry& g, float2* outO, double lam, const double* lam_dev, const float* dO,
                             const float2* vO, const int* predicate, hipStream_t s);
// out_P = sum of probe partials [+ lam * dP .* vP]; when a probe of M pixels gives fewer than
// PRB_WIDE blocks of 64 pixels and there are more than PRB_CHUNK segments, in two passes, the
// first summing chunks of PRB_CHUNK partials in place (the partials are consumed).
// prb_chunk_count: the number of chunks of the first pass, 0 for one pass.
constexpr int PRB_CHUNK = 32;
constexpr int PRB_WIDE = 128;
__host__ __device__ inline int prb_chunk_count(int M, int nseg) {
  return (nseg > PRB_CHUNK && (M + 63) / 64 < PRB_WIDE) ? (nseg + PRB_CHUNK - 1) / PRB_CHUNK : 0;
}
hipError_t launch_probe_reduce(const Geometry& g, float2* outP, double lam, const double* lam_dev, const float* dP,
                               const float2* vP, const int* predicate, hipStream_t s);
// both of the above in one launch (after the probe's first pass when it takes two); outP null:
// the object sum alone.  With pap, the launch's block b (probe blocks first, then the object
// tiles) also stores its part of the real inner product v.out at pap[4 b]; with pap_block,
// only the block *pap_block selects (0 object, 1 probe) contributes.
hipError_t launch_reduce_pair(const Geometry& g, float2* outO, float2* outP, double lam, const double* lam_dev,
                              const float* dO, const float* dP, const float2* vO, const float2* vP,
                              const int* predicate, hipStream_t s, double* pap = nullptr,
                              const int* pap_block = nullptr);
// number of blocks of launch_reduce_pair (the p.Ap parts it leaves)
inline int reduce_pair_blocks(const Geometry& g, bool probe) {
  return (probe ? (g.my * g.mx + 63) / 64 : 0) + g.otiles_x * g.otiles_y;
}
// out[j] = sum of the j-th entries of `count` double4 partials, j < nout (<= 4)
hipError_t launch_sum_partials(const double* partials, int count, double* out, int nout, hipStream_t s,
                               const int* pred = nullptr);
// paper's App. B diagonal from the stored traces
hipError_t launch_diag_paper(const Geometry& g, float* dO, float* dP, hipStream_t s, const int* pred = nullptr);
// dst[i] = src[i], i < n, unless *pred == 0 (copy_blocks(n) blocks)
hipError_t launch_copy(const float2* src, float2* dst, size_t n, const int* pred, hipStream_t s);
// up to MAX_COPIES independent copies in one launch (copy_blocks(n) blocks each)
hipError_t launch_copies(const CopyItem* items, int count, hipStream_t s);
hipError_t launch_sq_accum(const float2* u, float2* d, size_t n, float scale, int first, const int* pred,
                           hipStream_t s);
int copy_blocks(size_t n);
// batched forms (job tables in device memory)
// the object and probe sums of a batch in one launch (the probe part after a first pass over
// jb1, nb1 blocks: jobs with more than PRB_CHUNK segments, block1 their first, when nb1 > 0)
hipError_t launch_reduce_pair_batch(const RedJob* objjobs, const int* objjb, int nbo, const RedJob* prbjobs,
                                    const int* jb1, int nb1, const int* prbjb, int nbp, hipStream_t s);
hipError_t launch_sum_partials_batch(const RedJob* jobs, int njobs, int nout, hipStream_t s);
hipError_t launch_diag_paper_batch(const RedJob* objjobs, const int* objjb, int nbo, const RedJob* prbjobs,
                                   const int* prbjb, int nbp, hipStream_t s);
hipError_t launch_copy_batch(const CopyJob* jobs, const int* job_of_block, int nblocks, hipStream_t s);

}  // namespace ptlm
