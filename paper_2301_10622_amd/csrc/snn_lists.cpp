// Compaction: array containers next to the posting bitmaps.
//
// The paper keeps every inverted list I[j] as a compressed id list (Roaring,
// Section 4.1, Notes on Implementation), which chooses per chunk between a
// bitmap and a sorted array of offsets by density: an array while the chunk
// holds at most 1/16 of its possible ids. Here every coordinate keeps its
// bitmap (insert and delete flip bits in place), and a compaction gives the
// coordinates of density at most 1/16 an array container as well: per block
// of 1,024 slots, the block offsets of the coordinate's postings. Scoring such
// a coordinate then costs work per posting (a gather and an add per listed
// slot) instead of work per slot of every block. Blocks changed after the
// compaction are marked stale by the update kernels and read from the bitmaps
// until the next compaction; both readings add the same terms in the same
// order, so results do not depend on staleness.
//
// Which coordinates hold arrays (their class) does change how a score's terms
// are grouped -- the array terms are summed apart and added to the bitmap terms
// -- and so the last bits of a score. Two indexes with the same live documents
// and the same classes give identical results; snn_container_classes reads
// the classes and snn_compact can pin them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "snn.h"
#include "snn_host.h"

using namespace snn;

#define HIP_TRY(ix, call, what)                              \
  do {                                                       \
    hipError_t e__ = (call);                                 \
    if (e__ != hipSuccess) return (ix)->hip_fail(e__, what); \
  } while (0)

// Largest seg table a compaction builds (rows x (blocks + 1) x 4 bytes);
// coordinates past it keep their bitmap only.
static constexpr uint64_t kSegBudget = 4ull << 30;

snn_status snn_index::compact(const uint8_t *pinned) {
  const uint32_t dim = cfg.dim;
  const uint32_t nblk = cap >> 10;
  // every search and update in flight (on any stream) finishes before the
  // containers are replaced
  HIP_TRY(this, hipDeviceSynchronize(), "sync");
  std::vector<uint32_t> cnt(dim);
  {
    struct Counts {
      DevBuf b;
      ~Counts() { b.release(); }
    } cd;
    HIP_TRY(this, cd.b.ensure((size_t)dim * 4, stream), "compaction counts");
    HIP_TRY(this, launch_count_rows(dev, (uint32_t *)cd.b.p, stream), "count kernel");
    HIP_TRY(this, hipMemcpyAsync(cnt.data(), cd.b.p, (size_t)dim * 4, hipMemcpyDeviceToHost, stream),
            "counts readback");
    HIP_TRY(this, hipStreamSynchronize(stream), "sync");
  }
  // classes: an array container when the coordinate covers at most 1/16 of the
  // used blocks' slots (or as pinned); row 0 is shared by the array
  // coordinates without postings (all its segments empty)
  const uint64_t used = (uint64_t)((next_fresh + 1023u) >> 10) << 10;
  std::vector<uint32_t> crow_h(dim, kNoRow), row_coord;
  std::vector<uint64_t> rbase;
  std::vector<uint8_t> cls(dim, 0);
  uint64_t total = 0;
  const uint64_t max_rows = kSegBudget / ((uint64_t)(nblk + 1) * 4);
  for (uint32_t j = 0; j < dim; ++j) {
    const bool want = pinned ? pinned[j] != 0 : 16ull * cnt[j] <= used;
    if (!want) continue;
    if (cnt[j] == 0) {
      crow_h[j] = 0;
      cls[j] = 1;
      continue;
    }
    if (row_coord.size() + 2 > max_rows || total + cnt[j] > 0xFFFFFFF0ull) continue;  // over budget: bitmap
    crow_h[j] = (uint32_t)row_coord.size() + 1;
    cls[j] = 1;
    row_coord.push_back(j);
    rbase.push_back(total);
    total += cnt[j];
  }
  const uint32_t nrows = (uint32_t)row_coord.size();
  const size_t seg_bytes = (size_t)(nrows + 1) * (nblk + 1) * 4;
  // new buffers before the old ones go (a failure leaves the index as it was)
  struct Fresh {
    DevBuf seg, post, pu, pl, crow, aux;
    bool keep = false;
    ~Fresh() {
      aux.release();
      if (!keep) {
        seg.release();
        post.release();
        pu.release();
        pl.release();
        crow.release();
      }
    }
  } f;
  DevBuf &seg_n = f.seg, &post_n = f.post, &pu_n = f.pu, &pl_n = f.pl, &crow_n = f.crow, &aux = f.aux;
  const size_t vbytes = (dev.flags & kSketchBf16) ? 2 : 4;  // one bound, as the sketch holds it
  const bool lower = (dev.flags & kUpperOnly) == 0;
  HIP_TRY(this, seg_n.ensure(seg_bytes, stream), "array container offsets");
  HIP_TRY(this, post_n.ensure(total * 2 + 64, stream), "array containers");
  HIP_TRY(this, pu_n.ensure(total * vbytes + 64, stream), "array container bounds");
  if (lower) HIP_TRY(this, pl_n.ensure(total * vbytes + 64, stream), "array container bounds");
  HIP_TRY(this, crow_n.ensure((size_t)dim * 4, stream), "container rows");
  HIP_TRY(this, aux.ensure((size_t)nrows * 12 + 64, stream), "compaction rows");
  uint32_t *rc_d = (uint32_t *)aux.p;
  uint64_t *rb_d = (uint64_t *)((char *)aux.p + (((size_t)nrows * 4 + 15) / 16) * 16);
  HIP_TRY(this, hipMemcpyAsync(crow_n.p, crow_h.data(), (size_t)dim * 4, hipMemcpyHostToDevice, stream), "rows upload");
  if (nrows) {
    HIP_TRY(this, hipMemcpyAsync(rc_d, row_coord.data(), (size_t)nrows * 4, hipMemcpyHostToDevice, stream),
            "rows upload");
    HIP_TRY(this, hipMemcpyAsync(rb_d, rbase.data(), (size_t)nrows * 8, hipMemcpyHostToDevice, stream),
            "rows upload");
  }
  HIP_TRY(this, launch_fill_u32((uint32_t *)seg_n.p, 0u, nblk + 1, stream), "empty row");
  HIP_TRY(this,
          launch_build_lists(dev, nrows, rc_d, rb_d, (uint32_t *)seg_n.p + (nblk + 1), (uint16_t *)post_n.p, pu_n.p,
                             pl_n.p, stream),
          "list kernel");
  HIP_TRY(this, launch_fill_u32(dev.stale, 0u, nblk, stream), "stale flags");
  HIP_TRY(this, hipStreamSynchronize(stream), "sync");
  f.keep = true;
  lists_seg.release();
  lists_post.release();
  lists_pu.release();
  lists_pl.release();
  crow.release();
  lists_seg = seg_n;
  lists_post = post_n;
  lists_pu = pu_n;
  lists_pl = pl_n;
  crow = crow_n;
  dev.seg = (const uint32_t *)lists_seg.p;
  dev.post = (const uint16_t *)lists_post.p;
  dev.pu = lists_pu.p;
  dev.pl = lists_pl.p;
  classes = cls;
  array_coords = (uint32_t)std::count(cls.begin(), cls.end(), (uint8_t)1);
  free_slots.clear_stale();
  list_rows = nrows;
  list_postings = total;
  graphs.clear();  // captured launches hold the old containers
  return SNN_OK;
}

extern "C" snn_status snn_compact(snn_index *ix, const uint8_t *classes) {
  if (!ix) return SNN_E_INVALID;
  return ix->compact(classes);
}

extern "C" snn_status snn_container_classes(snn_index *ix, uint8_t *out) {
  if (!ix || !out) return SNN_E_INVALID;
  if (ix->classes.empty()) {
    std::fill(out, out + ix->cfg.dim, (uint8_t)0);
  } else {
    std::copy(ix->classes.begin(), ix->classes.end(), out);
  }
  return SNN_OK;
}
