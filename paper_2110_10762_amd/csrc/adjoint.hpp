#pragma once
#include "common.hpp"
namespace pr { struct AdjWork { int dummy; }; }
