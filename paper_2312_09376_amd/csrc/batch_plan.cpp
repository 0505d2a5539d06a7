// Host part of the batched solver's plan (rbt_batched_plan,
// rbt_batched_workspace_size): the workspace layout, the queue order and the
// header / descriptor-table image copied to the device. No device calls, so
// host builds of the batched kernel use the same plan.
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace rbt {

int check_batch_sizes(int64_t batch, const int64_t *n, const int64_t *nrhs) {
  if (batch < 0) return -1;
  if (batch > 0 && n == nullptr) return -2;
  if (batch > 0 && nrhs == nullptr) return -3;
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] < 0) return -2;
    if (nrhs[i] < 0) return -3;
    if (nrhs[i] > kSkinnyMax) return RBT_ERR_UNSUPPORTED;
  }
  return 0;
}

BatchPlanSizes batch_plan_sizes(int64_t batch, const int64_t *n, const int64_t *nrhs, int depth,
                                std::vector<BatchDesc> *desc) {
  BatchPlanSizes z{};
  z.f_off = align256(kBatchTableOffset + size_t(batch) * sizeof(BatchDesc));
  size_t f = 0, d = 0, f64 = 0;  // floats, doubles, fallback doubles
  std::vector<int64_t> order(batch);
  for (int64_t i = 0; i < batch; ++i) order[i] = i;
  // largest systems first (longest-processing-time order for the queue);
  // systems without work (n = 0 or nrhs = 0) last
  auto work_n = [&](int64_t i) { return nrhs[i] > 0 ? n[i] : int64_t(-1); };
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return work_n(a) > work_n(b); });
  if (desc) desc->resize(batch);
  for (int64_t t = 0; t < batch; ++t) {
    const int64_t i = order[t];
    if (desc) {
      BatchDesc &D = (*desc)[t];
      D = BatchDesc{};
      D.sys = i;
      D.n = n[i];
      D.nrhs = nrhs[i];
      D.f_off = int64_t(f);
      D.d_off = int64_t(d);
      D.f64_off = int64_t(f64);
    }
    f64 += align256(size_t(n[i]) * n[i] * sizeof(double)) / sizeof(double);
    f += align256(size_t(n[i]) * n[i] * sizeof(float)) / sizeof(float);
    d += align256(size_t(batched_sys_doubles(n[i], nrhs[i], depth)) * sizeof(double)) /
         sizeof(double);
  }
  z.d_off = align256(z.f_off + f * sizeof(float));
  z.f64_off = align256(z.d_off + d * sizeof(double));
  z.total = z.f64_off + f64 * sizeof(double);
  return z;
}

std::vector<char> batch_plan_image(int64_t batch, int depth, int prec, const BatchPlanSizes &z,
                                   const std::vector<BatchDesc> &desc) {
  std::vector<char> image(kBatchTableOffset + desc.size() * sizeof(BatchDesc), 0);
  BatchHeader h{};
  h.ticket = 0;
  h.batch = batch;
  h.depth = depth;
  h.prec = prec;
  h.f_off_bytes = int64_t(z.f_off);
  h.d_off_bytes = int64_t(z.d_off);
  h.total_bytes = int64_t(z.total);
  h.f64_off_bytes = int64_t(z.f64_off);
  std::memcpy(image.data(), &h, sizeof(h));
  if (!desc.empty())
    std::memcpy(image.data() + kBatchTableOffset, desc.data(), desc.size() * sizeof(BatchDesc));
  return image;
}

}  // namespace rbt
