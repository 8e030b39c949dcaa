// Exact labels (eq. 2) of single grid points in dyadic arithmetic on the input
// doubles: the arbiter of the points whose FP64 decision the classification
// kernels could not certify.  Plain C++ (host only, no HIP).
#pragma once

#include <cstdint>
#include <unordered_map>
#include <vector>

namespace eses {

// Atoms and concave probe positions of one molecule, on the host, with a
// uniform cell list over the centres for the neighbour queries.
class ExactMolecule {
  public:
    // centres [n][3], radii [n]; probes: ascending atom triples [nv][3] and
    // sides [nv] (+1: (p - c_a) . ((c_b - c_a) x (c_c - c_a)) > 0).
    ExactMolecule(const double *centres, const double *radii, int64_t n, double rho,
                  const int32_t *probe_atoms, const int8_t *probe_sign, int64_t nprobe);

    // 1 inside M, 0 outside, for the point x (three doubles).
    int label(const double x[3]);

  private:
    void near(const double x[3], double reach, std::vector<int> &out) const;
    const std::vector<int> &nbrs(int i);
    bool probe_within(int v, const double x[3]);
    bool face_candidate(int i, const double x[3]);
    bool circle_candidate(int i, int j, const double x[3]);

    std::vector<double> c_, r_;
    double rho_, smax_;
    int64_t n_;
    // cell list
    double lo_[3], cell_;
    int nc_[3];
    std::vector<int> cstart_, catom_;
    // probe positions per atom (each probe under its three atoms) and an
    // FP64 position for the reach filter
    std::vector<int> pa_;   // [nv][3]
    std::vector<int> ps_;   // [nv]
    std::vector<double> pp_;  // [nv][3] FP64 approximation
    std::vector<int> pstart_, plist_;
    std::unordered_map<int, std::vector<int>> nbr_;
};

// Sign of a dyadic expression, exposed for the CPU tests: sign of
// a sqrt(X) + b sqrt(Y) for doubles a, b, X >= 0, Y >= 0 (exactly).
int exact_sign_sqrt2(double a, double X, double b, double Y);

}  // namespace eses
