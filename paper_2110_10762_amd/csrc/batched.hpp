#pragma once
#include "common.hpp"
namespace pr { struct BatchWork { int dummy; }; }
struct pr_problem;
static int batched_solve_sync(pr_problem *, const double *, double *, pr_stats *);
