// Host-side logic of the serving loop, free of device code so that it can
// be tested on its own: the first-fit arena that admission allocates slot
// state from, and the error rule that picks Lanczos steps and probe counts.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace vne {

// First-fit allocator over [0, size): ranges are multiples of `align`, and
// a released range merges with free neighbours.
class Arena {
public:
    explicit Arena(uint64_t size = 0, uint64_t align = 256) { reset(size, align); }
    void reset(uint64_t size, uint64_t align = 256);
    // lowest free range that holds `bytes` (rounded up to align); false if none
    bool alloc(uint64_t bytes, uint64_t *off);
    // a range returned by alloc; returns false for an unknown offset
    bool release(uint64_t off);
    uint64_t size() const { return size_; }
    uint64_t in_use() const { return used_; }
    uint64_t largest_free() const;
    uint64_t round(uint64_t bytes) const { return (bytes + align_ - 1) / align_ * align_; }
    size_t free_ranges() const { return free_.size(); }

private:
    uint64_t size_ = 0, align_ = 256, used_ = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    std::map<uint64_t, uint64_t> live_;   // offset -> length
};

// Lanczos steps for a quadrature error of at most share * rel_eps * s_lower
// per quadratic form: Proposition 4.4 (polynomial Krylov space) with the
// gamma = 0 bound of Remark 2.3 at degree 2k - 1,
//     |psi - psi_k| <= 2 ||c||^2 lambda_max / (4 ((2k - 1)^2 - 1)),
// smallest k >= 2 that meets the target, at most k_max.  Returns k_max when
// the target is not positive.
int32_t plan_steps(double norm2, double lambda_max, double s_lower, double rel_eps, double share,
                   int32_t k_max);

// Probe count for a sampling error of share * rel_eps * s_hat at z standard
// errors: ceil((z sigma / (share rel_eps s_hat))^2), clamped to [n_min, n_max].
int32_t plan_probes(double s_hat, double sigma, double rel_eps, double share, double z, int32_t n_min,
                    int32_t n_max);

}  // namespace vne
