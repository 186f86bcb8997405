// Host-side serving logic: arena allocator and error rule.
#include "serve_host.h"

#include <algorithm>
#include <cmath>
#include <iterator>

#include "vne.h"

namespace vne {

void Arena::reset(uint64_t size, uint64_t align) {
    align_ = align ? align : 1;
    size_ = size / align_ * align_;
    used_ = 0;
    free_.clear();
    live_.clear();
    if (size_) free_[0] = size_;
}

bool Arena::alloc(uint64_t bytes, uint64_t *off) {
    const uint64_t need = round(std::max<uint64_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second < need) continue;
        const uint64_t o = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[o + need] = len - need;
        live_[o] = need;
        used_ += need;
        *off = o;
        return true;
    }
    return false;
}

bool Arena::release(uint64_t off) {
    auto lv = live_.find(off);
    if (lv == live_.end()) return false;
    uint64_t o = off, len = lv->second;
    live_.erase(lv);
    used_ -= len;
    auto next = free_.lower_bound(o);
    if (next != free_.end() && next->first == o + len) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == o) {
            prev->second += len;
            return true;
        }
    }
    free_[o] = len;
    return true;
}

uint64_t Arena::largest_free() const {
    uint64_t m = 0;
    for (const auto &kv : free_) m = std::max(m, kv.second);
    return m;
}

int32_t plan_steps(double norm2, double lambda_max, double s_lower, double rel_eps, double share,
                   int32_t k_max) {
    const double target = share * rel_eps * s_lower;
    if (!(target > 0.0) || k_max < 2) return std::max<int32_t>(k_max, 1);
    auto bound = [&](int k) {
        const double d = 2.0 * k - 1.0;
        return 2.0 * norm2 * lambda_max / (4.0 * (d * d - 1.0));
    };
    // (2k-1)^2 >= 1 + norm2 lambda_max / (2 target), then fix rounding
    const double q = 1.0 + norm2 * lambda_max / (2.0 * target);
    double k0 = std::ceil((std::sqrt(q) + 1.0) / 2.0);
    if (!(k0 < (double)k_max)) k0 = k_max;
    int32_t k = std::max<int32_t>(2, (int32_t)k0);
    while (k > 2 && bound(k - 1) <= target) --k;
    while (k < k_max && bound(k) > target) ++k;
    return k;
}

int32_t plan_probes(double s_hat, double sigma, double rel_eps, double share, double z, int32_t n_min,
                    int32_t n_max) {
    const double target = share * rel_eps * std::fabs(s_hat);
    if (!(target > 0.0)) return n_max;
    const double n = std::ceil(std::pow(z * sigma / target, 2.0));
    if (!(n < (double)n_max)) return n_max;
    return std::max<int32_t>(n_min, (int32_t)n);
}

}  // namespace vne

extern "C" int32_t vne_plan_steps(double norm2, double lambda_max, double s_lower, double rel_eps, double share,
                                  int32_t k_max) {
    return vne::plan_steps(norm2, lambda_max, s_lower, rel_eps, share, k_max);
}

extern "C" int32_t vne_plan_probes(double s_hat, double sigma, double rel_eps, double share, double z,
                                   int32_t n_min, int32_t n_max) {
    return vne::plan_probes(s_hat, sigma, rel_eps, share, z, n_min, n_max);
}
