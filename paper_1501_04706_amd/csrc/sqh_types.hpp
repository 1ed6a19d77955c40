// Data layout shared by the device kernels and the host driver of libsqh.
#pragma once
#include <stdint.h>

namespace sqh {

// Per point set: the seeds of the first split (section 4.3: leftmost and
// rightmost points; here lexicographic, so ties in x are decided by y) and
// the farthest point on each side of the line through them.
struct SetInfo {
    float ax, ay, bx, by;      // A = lexmin, B = lexmax position
    int aid, bid;              // their indices within the set (lowest at the position)
    int apos, bpos;            // their global positions
    float clx, cly, cux, cuy;  // farthest points below (lower) and above (upper) A->B
    int clid, cuid;            // their indices within the set
    int n_lo, n_up;            // points strictly right of A->B / of B->A
};

// One segment (paper section 2; Table 1 keeps the same information per
// point in head[], keys[] and first_pts[]): the directed hull edge A->B, the
// farthest of its points C (section 4.4.1), and the slots
// [off, off + len) of its points in the survivor buffer. Child records
// produced by a pass use the same layout (len == 0: the edge is final).
struct Seg {
    float ax, ay, bx, by;
    float cx, cy;
    int off, len;
};

}  // namespace sqh
