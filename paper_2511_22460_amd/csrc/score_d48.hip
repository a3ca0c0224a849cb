// k_score and k_rescore at embedding width 48.
#include "score.h"

namespace ebr {
template void launch_score_d<48>(const ScoreArgs&, int, int, dim3, hipStream_t);
template void launch_rescore_d<48>(const RescoreArgs&, int, hipStream_t);
}  // namespace ebr
