"""Host Jacobi eigensolver of the coarsest deflation setup, against numpy.

csrc/herm_eig.h is plain C++; a small driver compiled with g++ reads a
Hermitian matrix, and its eigenvalues must equal numpy.linalg.eigh's, its
eigenvectors must satisfy H v = lambda v and be orthonormal (to 1e-12 of
the matrix norm), on random, degenerate and diagonal inputs.
"""
import os
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1011_2775_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include "herm_eig.h"
int main() {
  int m;
  if (scanf("%d", &m) != 1) return 1;
  std::vector<std::complex<double>> H((size_t)m * m);
  for (auto& h : H) { double re, im; if (scanf("%lf %lf", &re, &im) != 2) return 1; h = {re, im}; }
  std::vector<double> ev;
  std::vector<std::complex<double>> V;
  wcmg::hermitian_eig(H, m, ev, V);
  for (double e : ev) printf("%.17g\n", e);
  for (auto& v : V) printf("%.17g %.17g\n", v.real(), v.imag());
  return 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("eig")
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(d / "drv.cpp"), "-o", str(exe)], check=True)
    return str(exe)


def run(exe, H):
    m = H.shape[0]
    inp = "%d\n" % m + "\n".join("%.17g %.17g" % (z.real, z.imag) for z in H.reshape(-1))
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    ev = np.array([float(x) for x in out[:m]])
    V = np.array([complex(*map(float, l.split())) for l in out[m:m + m * m]]).reshape(m, m)
    return ev, V


@pytest.mark.parametrize("m,kind", [(5, "random"), (48, "random"), (96, "random"), (12, "degenerate"),
                                    (7, "diagonal"), (1, "random")])
def test_hermitian_eig(driver, m, kind):
    rng = np.random.default_rng(m)
    if kind == "diagonal":
        H = np.diag(rng.standard_normal(m)).astype(np.complex128)
    else:
        A = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
        H = A @ A.conj().T if kind == "random" else None
        if kind == "degenerate":
            Qm, _ = np.linalg.qr(A)
            H = Qm @ np.diag(np.repeat([1.0, 2.0, 5.0], m // 3)) @ Qm.conj().T
    ev, V = run(driver, H)
    scale = np.linalg.norm(H)
    assert np.allclose(ev, np.linalg.eigvalsh(H), atol=1e-12 * scale, rtol=0)
    assert np.abs(H @ V - V * ev).max() <= 1e-12 * scale
    assert np.abs(V.conj().T @ V - np.eye(m)).max() <= 1e-12
