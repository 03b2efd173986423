// Filter GEMM instantiations for the widest tiles (9 and 10 16-column
// blocks per wave), built like the others with the VGPR form of MFMA (see
// k_filter_kern.h).
#include "k_filter_kern.h"

namespace chase {

void launch_filter_wide(const FilterPlan &p, const Z *H, int64_t ldh, int N,
                        const Z *Y, int64_t ldy, const Z *X, int64_t ldx, Z *W,
                        int64_t ldw, int n, double a, double b, double g, Z *part,
                        hipStream_t s) {
    using namespace filter_detail;
    if (p.wn == 9) launch_wn<9>(p, H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, part, s);
    else if (p.wn == 10) launch_wn<10>(p, H, ldh, N, Y, ldy, X, ldx, W, ldw, n, a, b, g, part, s);
    else throw Error(7, "launch_filter_wide: bad tile width");
}

void launch_filter_group_wide(int wn, const FilterPlan *plans, const FilterCall *calls,
                              int count, hipStream_t s) {
    using namespace filter_detail;
    if (wn == 9) launch_group_wn<9>(plans, calls, count, s);
    else if (wn == 10) launch_group_wn<10>(plans, calls, count, s);
    else throw Error(7, "launch_filter_group_wide: bad tile width");
}

}  // namespace chase
