// Host check of the register-resident FFT arithmetic (paper_2207_09028_amd/csrc/regfft.hpp):
// the H-point in-register DFTs and the two-lane DIT / DIF line transforms, with both
// lanes of a pair emulated on the CPU, against a direct O(N^2) DFT in long double.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "regfft.hpp"

using namespace occrik;
typedef std::complex<long double> CL;

static std::vector<CL> direct(const std::vector<CL>& x, int dir) {
    const int n = (int)x.size();
    std::vector<CL> X(n);
    for (int k = 0; k < n; ++k) {
        CL s = 0;
        for (int j = 0; j < n; ++j) {
            const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)((long long)j * k % n) / n;
            s += x[j] * CL(std::cos(a), dir * std::sin(a));
        }
        X[k] = s;
    }
    return X;
}

template <typename T, int H, int DIR>
static double check_reg(std::mt19937& g) {
    std::normal_distribution<double> nd;
    std::vector<CL> x(H);
    cplx<T> v[H];
    for (int i = 0; i < H; ++i) {
        x[i] = CL(nd(g), nd(g));
        v[i].x = (T)x[i].real();
        v[i].y = (T)x[i].imag();
        x[i] = CL((long double)v[i].x, (long double)v[i].y);
    }
    reg_dft<T, H, DIR>(v);
    const auto X = direct(x, DIR);
    double e = 0, m = 0;
    for (int k = 0; k < H; ++k) {
        e = std::fmax(e, (double)std::abs(CL(v[k].x, v[k].y) - X[k]));
        m = std::fmax(m, (double)std::abs(X[k]));
    }
    return e / m;
}

template <typename T, int N, int DIR>
static double check_lines(std::mt19937& g) {
    constexpr int H = N / 2;
    std::normal_distribution<double> nd;
    std::vector<CL> x(N);
    for (auto& c : x) c = CL((T)nd(g), (T)nd(g));
    const auto X = direct(x, DIR);
    double m = 0;
    for (auto& c : X) m = std::fmax(m, (double)std::abs(c));
    double e = 0;
    // DIT: interleaved in -> blocked out
    {
        cplx<T> a[2][H], send[2][H / 2];
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < H; ++i) {
                a[s][i].x = (T)x[2 * i + s].real();
                a[s][i].y = (T)x[2 * i + s].imag();
            }
        for (int s = 0; s < 2; ++s) dit_local<T, N, DIR>(a[s], s);
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < H / 2; ++i) send[s][i] = a[s][H / 2 + i];
        for (int s = 0; s < 2; ++s) dit_combine<T, N>(a[s], send[1 - s], s);
        for (int s = 0; s < 2; ++s)
            for (int mm = 0; mm < H; ++mm) {
                const int k = blocked_index(mm, s, H);
                e = std::fmax(e, (double)std::abs(CL(a[s][mm].x, a[s][mm].y) - X[k]));
            }
    }
    // DIF: blocked in -> interleaved out
    {
        cplx<T> a[2][H], send[2][H / 2];
        for (int s = 0; s < 2; ++s)
            for (int mm = 0; mm < H; ++mm) {
                const int i = blocked_index(mm, s, H);
                a[s][mm].x = (T)x[i].real();
                a[s][mm].y = (T)x[i].imag();
            }
        for (int s = 0; s < 2; ++s) dif_local<T, N, DIR>(a[s], s);
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < H / 2; ++i) send[s][i] = a[s][H / 2 + i];
        for (int s = 0; s < 2; ++s) dif_combine<T, N, DIR>(a[s], send[1 - s], s);
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < H; ++k)
                e = std::fmax(e, (double)std::abs(CL(a[s][k].x, a[s][k].y) - X[2 * k + s]));
    }
    return e / m;
}

int main() {
    std::mt19937 g(1234);
    int bad = 0;
    auto report = [&](const char* what, int n, double e, double tol) {
        const bool ok = e < tol;
        bad += !ok;
        std::printf("%-14s N=%2d rel err %.3e %s\n", what, n, e, ok ? "ok" : "FAIL");
    };
#define REG(H) report("reg64 fwd", H, check_reg<double, H, -1>(g), 1e-14); \
               report("reg64 inv", H, check_reg<double, H, +1>(g), 1e-14); \
               report("reg32 fwd", H, check_reg<float, H, -1>(g), 2e-6);
    REG(2) REG(3) REG(4) REG(5) REG(6) REG(8) REG(9) REG(10) REG(12) REG(15) REG(16) REG(18) REG(20) REG(24)
#define LIN(N) report("lines64 fwd", N, check_lines<double, N, -1>(g), 1e-14); \
               report("lines64 inv", N, check_lines<double, N, +1>(g), 1e-14); \
               report("lines32 fwd", N, check_lines<float, N, -1>(g), 2e-6);
    LIN(24) LIN(32) LIN(36) LIN(40) LIN(48)
    return bad ? 1 : 0;
}
