// Host harness for the balanced domain order (letkf::balanced_order, host
// code of libletkf.so): reads "n num_cu resident" and n costs from stdin,
// prints the XCD order and the balanced order, one line each.  Needs no GPU.
#include <cstdio>
#include <vector>

#include "internal.hpp"

int main() {
  int n = 0, num_cu = 0, resident = 0;
  if (std::scanf("%d %d %d", &n, &num_cu, &resident) != 3 || n < 1) return 2;
  std::vector<double> cost(n);
  for (double& c : cost)
    if (std::scanf("%lf", &c) != 1) return 2;
  letkf::Problem P;
  P.n_dom = n;
  const std::vector<int32_t> xcd = letkf::domain_order(P, LETKF_ORDER_XCD);
  const std::vector<int32_t> bal = letkf::balanced_order(P, cost, num_cu, resident);
  for (int32_t v : xcd) std::printf("%d ", v);
  std::printf("\n");
  for (int32_t v : bal) std::printf("%d ", v);
  std::printf("\n");
  return 0;
}
