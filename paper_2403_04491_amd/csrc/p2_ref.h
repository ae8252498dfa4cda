// Reference integrals of the Lagrange bases of degree 1 and 2 on a simplex, host side.
//
// On an m-simplex with barycentric coordinates lambda_0..lambda_m the P2 basis is
// lambda_a (2 lambda_a - 1) at the vertices, then 4 lambda_a lambda_b at the edges,
// (a, b) with a < b in lexicographic order (Sec. "Spatial discretization": Lagrange
// elements of degree p on the simplices).  Products of basis functions and of their
// derivatives in lambda are polynomials in lambda, integrated exactly with
//   int prod lambda_a^{p_a} = m! |T| prod p_a! / (m + sum p_a)!.
// Plain C++ (no HIP), so that it can be compiled on its own for host checks.
#pragma once

#include <array>
#include <cstdint>
#include <map>
#include <vector>

namespace knp {
namespace p2 {

// A polynomial in at most 4 barycentric coordinates: exponent vector -> coefficient.
using Expo = std::array<int, 4>;
using Poly = std::map<Expo, double>;

inline Poly pmul(const Poly &p, const Poly &q) {
    Poly r;
    for (const auto &x : p)
        for (const auto &y : q) {
            Expo e;
            for (int k = 0; k < 4; ++k) e[k] = x.first[k] + y.first[k];
            r[e] += x.second * y.second;
        }
    return r;
}

// derivative with respect to lambda_v
inline Poly pdiff(const Poly &p, int v) {
    Poly r;
    for (const auto &x : p) {
        if (x.first[v] == 0) continue;
        Expo e = x.first;
        e[v] -= 1;
        r[e] += double(x.first[v]) * x.second;
    }
    return r;
}

inline double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// integral over an m-simplex divided by its measure
inline double pint(const Poly &p, int m) {
    double s = 0.0;
    for (const auto &x : p) {
        double num = factorial(m);
        int deg = 0;
        for (int k = 0; k < 4; ++k) {
            num *= factorial(x.first[k]);
            deg += x.first[k];
        }
        s += x.second * num / factorial(m + deg);
    }
    return s;
}

// the Lagrange basis of degree 1 (the barycentric coordinates) or 2 (m + 1 vertex
// functions, then the edge functions) on an m-simplex
inline std::vector<Poly> basis(int m, int order = 2) {
    const int n = m + 1;
    std::vector<Poly> out;
    if (order == 1) {
        for (int a = 0; a < n; ++a) {
            Poly p;
            Expo e{0, 0, 0, 0};
            e[a] = 1;
            p[e] = 1.0;
            out.push_back(p);
        }
        return out;
    }
    for (int a = 0; a < n; ++a) {
        Poly p;
        Expo e2{0, 0, 0, 0}, e1{0, 0, 0, 0};
        e2[a] = 2;
        e1[a] = 1;
        p[e2] = 2.0;
        p[e1] = -1.0;
        out.push_back(p);
    }
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b) {
            Poly p;
            Expo e{0, 0, 0, 0};
            e[a] = e[b] = 1;
            p[e] = 4.0;
            out.push_back(p);
        }
    return out;
}

// Reference tensors of the element on a d-simplex (n = d+1 coordinates, nb nodes), per
// unit measure:  M[a][b] = int phi_a phi_b;  S[a][b][i][j] = int d_i phi_a d_j phi_b;
// W[c][a][b][i][j] = int phi_c d_i phi_a d_j phi_b (d_i: derivative in lambda_i).  The
// physical stiffness is then |T| sum_ij G_ij S[a][b][i][j] with G_ij = grad lambda_i .
// grad lambda_j.  Facet tensors on the (d-1)-simplex: F2[a][b] = int phi_a phi_b,
// F3[a][b][c] = int phi_a phi_b phi_c.  Flat, row-major.
struct RefTensors {
    int d = 0, n = 0, nb = 0, nf = 0;   // coordinates, element nodes, facet nodes
    std::vector<double> M, S, W, F2, F3;
};

inline RefTensors reference_tensors(int d, int order = 2) {
    RefTensors t;
    t.d = d;
    t.n = d + 1;
    const std::vector<Poly> B = basis(d, order);
    t.nb = int(B.size());
    const int n = t.n, nb = t.nb;
    std::vector<std::vector<Poly>> dB(nb);
    for (int a = 0; a < nb; ++a)
        for (int i = 0; i < n; ++i) dB[a].push_back(pdiff(B[a], i));
    t.M.assign(size_t(nb) * nb, 0.0);
    t.S.assign(size_t(nb) * nb * n * n, 0.0);
    t.W.assign(size_t(nb) * nb * nb * n * n, 0.0);
    for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
            t.M[size_t(a) * nb + b] = pint(pmul(B[a], B[b]), d);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const Poly pij = pmul(dB[a][i], dB[b][j]);
                    t.S[((size_t(a) * nb + b) * n + i) * n + j] = pint(pij, d);
                    for (int c = 0; c < nb; ++c)
                        t.W[(((size_t(c) * nb + a) * nb + b) * n + i) * n + j] = pint(pmul(B[c], pij), d);
                }
        }
    const std::vector<Poly> Fb = basis(d - 1, order);
    t.nf = int(Fb.size());
    const int nf = t.nf;
    t.F2.assign(size_t(nf) * nf, 0.0);
    t.F3.assign(size_t(nf) * nf * nf, 0.0);
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            const Poly ab = pmul(Fb[a], Fb[b]);
            t.F2[size_t(a) * nf + b] = pint(ab, d - 1);
            for (int c = 0; c < nf; ++c) t.F3[(size_t(a) * nf + b) * nf + c] = pint(pmul(ab, Fb[c]), d - 1);
        }
    return t;
}

}  // namespace p2
}  // namespace knp
