// Prints w(z) from faddeeva.hpp for z read as "x y" lines on stdin, one "re im" line each.
#include <cstdio>

#include "faddeeva.hpp"

int main() {
    double x, y;
    while (std::scanf("%lf %lf", &x, &y) == 2) {
        double wr, wi;
        occrik::fad::faddeeva(x, y, wr, wi);
        std::printf("%.17e %.17e\n", wr, wi);
    }
    return 0;
}
